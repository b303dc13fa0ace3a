"""The GPU partitioner at the variable-partition workload's full size (three
uint32 columns of 10^8 values, tau 0.03, merge passes until one merges
nothing), against the oracle where the oracle can follow:

* on sampled windows: a boundary the final partitioning keeps was kept by
  every merge pass and begins a split partition, so the split and every
  pass restart their state there, and the oracle's greedy run on the window
  alone must give exactly the GPU's starts inside it (windows chosen among
  short partitions, where the oracle's merge is fast);
* at every size: starts increase from 0 to n, no partition exceeds the cap,
  and the merge's fixed point holds on sampled neighbours (merging a pair
  would not make it strictly smaller, or would exceed the cap)."""
from __future__ import annotations

import numpy as np
import pytest

from paper_2306_15374_amd import workloads as W

pytestmark = pytest.mark.gpu

N = 100_000_000
TAU = 0.03
CAP = 1 << 20


@pytest.fixture(scope="module")
def torch():
    import torch as T
    if not T.cuda.is_available():
        pytest.skip("no GPU")
    return T


@pytest.fixture(scope="module")
def codec(torch):
    import paper_2306_15374_amd as P
    c = P.Codec(0)
    yield c
    c.close()


def windows(starts: np.ndarray, rng, count: int = 3, lo: int = 30_000, hi: int = 120_000,
            longest: int = 6000):
    """Up to `count` windows [b, e) of kept boundaries spanning lo..hi values
    whose partitions all hold at most `longest` values."""
    lens = np.diff(starts.astype(np.int64))
    out = []
    for _ in range(400):
        if len(out) == count:
            break
        i = int(rng.integers(0, len(lens)))
        j, span = i, 0
        while j < len(lens) and span < lo and lens[j] <= longest:
            span += int(lens[j])
            j += 1
        if lo <= span <= hi and all(b >= int(starts[j]) or e <= int(starts[i]) for b, e in out):
            out.append((int(starts[i]), int(starts[j])))
    return out


@pytest.mark.parametrize("kind", ["sorted_normal", "piecewise_linear", "constant_runs"])
def test_full_size_partition(torch, codec, ref, kind):
    gen = {"sorted_normal": W.sorted_normal, "piecewise_linear": W.piecewise_linear,
           "constant_runs": W.constant_runs}[kind]
    seed = W.C3_SEEDS[["sorted_normal", "piecewise_linear", "constant_runs"].index(kind)]
    print(f"[full] {kind}: drawing {N} values", flush=True)
    col = gen(N, seed)
    starts = codec.partition(torch.from_numpy(col).cuda(), tau=TAU)
    print(f"[full] {kind}: {len(starts) - 1} partitions", flush=True)
    s = starts.astype(np.int64)
    assert s[0] == 0 and s[-1] == N and bool(np.all(np.diff(s) > 0))
    assert int(np.diff(s).max()) <= CAP
    rng = np.random.default_rng(5)
    # the merge's fixed point on sampled neighbours
    m = len(s) - 1
    for k in rng.choice(np.arange(1, m), size=min(m - 1, 3000), replace=False):
        a, b, c = int(s[k - 1]), int(s[k]), int(s[k + 1])
        if c - a > CAP:
            continue
        merged = ref.partition_cost_bytes(col[a:c], 0, c - a)
        apart = (ref.partition_cost_bytes(col[a:b], 0, b - a)
                 + ref.partition_cost_bytes(col[b:c], 0, c - b))
        assert merged >= apart, f"{kind}: neighbours at {a}, {b}, {c} would merge"
    # exact parity on windows
    wins = windows(starts, rng)
    assert wins, f"{kind}: no window of short partitions found"
    for b, e in wins:
        print(f"[full] {kind}: oracle on [{b}, {e})", flush=True)
        expect = ref.partition_greedy(np.ascontiguousarray(col[b:e]), tau=TAU).astype(np.int64) + b
        got = s[(s >= b) & (s <= e)]
        assert np.array_equal(got, expect), (
            f"{kind}: window [{b}, {e}): {len(got) - 1} GPU partitions, {len(expect) - 1} oracle")
