"""GPU variable-length partitioner (section 3.2.2) against the oracle's
greedy split + merge scan: identical partition starts (integer work:
exact), on the column shapes of the variable-partition workloads, both
widths, first differences beyond 64 bits, several thresholds and caps,
columns longer than one 2^20-value split segment, partitions crossing
segment boundaries, and merge chains across the speculative chunks (256
partitions) and fix-up groups (64 chunks) of the merge scan."""
from __future__ import annotations

import sys

import numpy as np
import pytest

import paper_2306_15374_amd as P
from paper_2306_15374_amd import workloads as W

pytestmark = pytest.mark.gpu


def log(msg: str):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as T
    if not T.cuda.is_available():
        pytest.skip("no GPU")
    return T


@pytest.fixture(scope="module")
def codec(torch):
    c = P.Codec(0)
    yield c
    c.close()


def check(torch, codec, ref, col: np.ndarray, name: str, **kw):
    log(f"[partition] {name}: n={len(col)} dtype={col.dtype} {kw}")
    expect = ref.partition_greedy(col, **kw)
    got = codec.partition(torch.from_numpy(np.ascontiguousarray(col)).cuda(), **kw)
    assert len(got) == len(expect), f"{name}: m {len(got) - 1} != {len(expect) - 1}"
    if not np.array_equal(got, expect):
        bad = np.flatnonzero(got != expect)
        raise AssertionError(f"{name}: {len(bad)} starts differ, first at {bad[0]}: "
                             f"{got[bad[0]]} != {expect[bad[0]]}")
    return got


@pytest.mark.parametrize("kind", ["sorted_normal", "piecewise_linear", "constant_runs"])
def test_workload_shapes(torch, codec, ref, kind):
    n = 200_000
    col = {"sorted_normal": lambda: W.sorted_normal(n, W.C3_SEEDS[0]),
           "piecewise_linear": lambda: W.piecewise_linear(n, W.C3_SEEDS[1], segments=50),
           "constant_runs": lambda: W.constant_runs(n, W.C3_SEEDS[2])}[kind]()
    starts = check(torch, codec, ref, col, kind)
    # the GPU starts encode to the oracle's bytes and decode back
    blob = codec.encode(torch.from_numpy(col).cuda(), starts=starts)
    assert np.array_equal(blob.cpu().numpy(), ref.encode(col, starts=starts))


def test_thresholds_caps_and_widths(torch, codec, ref):
    rng = np.random.default_rng(71)
    noise = W.linear_noise(50_000, 72)
    keys32 = W.lognormal_keys(50_000, 73, np.uint32)
    check(torch, codec, ref, noise, "noise tau 0", tau=0.0)
    check(torch, codec, ref, noise, "noise tau 0.15", tau=0.15)
    check(torch, codec, ref, noise, "noise sm 64", sm_bits=64)
    check(torch, codec, ref, keys32, "keys u32 cap 1000", max_len=1000)
    check(torch, codec, ref, keys32, "keys u32 cap 1", max_len=1)
    check(torch, codec, ref, keys32[:3000], "keys u32 cap 7 tau 0.05", max_len=7, tau=0.05)
    # first differences spanning more than 64 bits (v alternating near 0 and 2^64)
    wide = rng.integers(0, 2**64 - 1, 20_000, dtype=np.uint64, endpoint=True)
    wide[::3] = rng.integers(0, 16, len(wide[::3]), dtype=np.uint64)
    wide[1::3] = np.uint64(2**64 - 1) - rng.integers(0, 16, len(wide[1::3]), dtype=np.uint64)
    check(torch, codec, ref, wide, "65-bit differences")
    mixed = np.concatenate([W.piecewise_linear(30_000, 74, segments=20),
                            rng.integers(0, 2**40, 5_000, dtype=np.uint64),
                            np.full(10_000, 123456789, dtype=np.uint64)])
    check(torch, codec, ref, mixed, "mixed regimes")


def test_merge_pass_limits(torch, codec, ref):
    col = W.piecewise_linear(60_000, 75, segments=30)
    for r in (1, 2, 3):
        check(torch, codec, ref, col, f"max_passes {r}", max_passes=r)


def test_merge_chains_across_chunks_and_groups(torch, codec, ref):
    """tau = 0 splits noisy columns into partitions of two or three values,
    about 150,000 of them: the merge scan then runs chains of merges across
    its 256-partition chunks and 64-chunk groups (until widening the
    residuals by a bit costs more than a record), over several passes."""
    rng = np.random.default_rng(88)
    poly = W.piecewise_linear(300_000, 91, segments=150).astype(np.uint64)
    check(torch, codec, ref, poly, "polyline u64 tau 0", tau=0.0)
    poly32 = W.piecewise_linear(300_000, 92, segments=150)
    check(torch, codec, ref, poly32, "polyline u32 tau 0, sm 96", tau=0.0, sm_bits=96)
    check(torch, codec, ref, poly, "polyline tau 0, one pass", tau=0.0, max_passes=1)
    noise = (np.arange(300_000, dtype=np.uint64) * np.uint64(9)
             + rng.integers(0, 8, 300_000, dtype=np.uint64))
    check(torch, codec, ref, noise, "noise tau 0, cap 500", tau=0.0, max_len=500)
    runs = W.constant_runs(300_000, 89, mean_run=5)
    check(torch, codec, ref, runs, "short runs tau 0", tau=0.0)


def test_merge_chains_wide_values(torch, codec, ref):
    """Long runs of merges (tau = 0 splits into partitions of two values,
    the scan merges them back into partitions of thousands) on 64-bit
    values whose spread needs the 64-bit turn tests of the partition's hulls
    (2^38), the 128-bit ones (2^58), and steep lines whose largest
    prediction reaches 2^33, where the hull range test hands every batch to
    a scan of all the values."""
    rng = np.random.default_rng(90)
    n = 60_000
    base = W.piecewise_linear(n, 93, segments=20).astype(np.uint64)
    check(torch, codec, ref, base * np.uint64(1 << 20) + rng.integers(0, 1 << 20, n, dtype=np.uint64),
          "polyline x 2^20 (spread 2^38)", tau=0.0)
    check(torch, codec, ref, base * np.uint64(1 << 40) + rng.integers(0, 1 << 40, n, dtype=np.uint64),
          "polyline x 2^40 (spread 2^58)", tau=0.0)
    steep = np.arange(n, dtype=np.uint64) * np.uint64(1 << 22) + rng.integers(0, 1 << 12, n,
                                                                            dtype=np.uint64)
    check(torch, codec, ref, steep, "steep line (predictions beyond 2^31)", tau=0.0)
    check(torch, codec, ref, steep, "steep line, one pass, cap 3000", tau=0.0, max_passes=1,
          max_len=3000)


def test_cap_counts_from_the_partition_start(torch, codec, ref):
    """One line cut by the cost at 1000, then 2^20 + 5000 values of another
    line: the cap cuts at 1000 + 2^20, inside the second split segment."""
    n2 = (1 << 20) + 5000
    col = np.concatenate([np.arange(1000, dtype=np.uint64) * np.uint64(3),
                          np.uint64(10**9) + np.arange(n2, dtype=np.uint64) * np.uint64(3)])
    got = check(torch, codec, ref, col, "line across a segment boundary")
    assert list(got) == [0, 1000, 1000 + (1 << 20), len(col)]


def test_tiny_columns(torch, codec, ref):
    for n in (1, 2, 3, 63, 64, 65, 127, 4097):
        col = W.lognormal_keys(n, 76 + n)
        check(torch, codec, ref, col, f"n={n}")
    empty = codec.partition(torch.zeros(0, dtype=torch.int64, device="cuda"))
    assert list(empty) == [0]


def test_longer_than_one_segment(torch, codec, ref):
    """Several 2^20-value split segments, a ragged last one, and merges that
    would cross a segment boundary only when the union fits 2^20."""
    n = 2 * (1 << 20) + 70_001
    col = W.sorted_normal(n, 77)
    check(torch, codec, ref, col, "sorted normal, 3 segments")
    runs = W.constant_runs(n, 78)
    check(torch, codec, ref, runs, "constant runs, 3 segments")


def test_starting_positions(torch, codec, ref):
    """With starting partitions (section 3.2.2, runs of smallest
    second-order delta) the split begins a partition at the first value of
    each and includes its other values without the cost test: identical
    starts on the workload shapes, both widths, a column whose smallest
    second-order delta is 3 (one starting partition over the whole column),
    differences beyond 64 bits, tiny columns and several 2^20-value split
    segments (starting partitions across segment and sub-chunk
    boundaries)."""
    rng = np.random.default_rng(81)
    n = 200_000
    for kind, col in [("sorted_normal", W.sorted_normal(n, W.C3_SEEDS[0])),
                      ("piecewise_linear", W.piecewise_linear(n, W.C3_SEEDS[1], segments=50)),
                      ("constant_runs", W.constant_runs(n, W.C3_SEEDS[2])),
                      ("noise u64", W.linear_noise(100_000, 82)),
                      ("keys u32", W.lognormal_keys(100_000, 83, np.uint32))]:
        starts = check(torch, codec, ref, col, f"{kind} with starting positions",
                       start_positions=True, tau=0.05)
        assert set(int(p) for p in ref.start_positions(col)) <= set(
            int(s) for s in ref.partition_split(col, tau=0.05, start_positions=True))
        check(torch, codec, ref, col[:60_000], f"{kind} with starting positions, tau 0",
              start_positions=True, tau=0.0)
        if kind == "constant_runs":
            blob = codec.encode(torch.from_numpy(col).cuda(), starts=starts)
            assert np.array_equal(blob.cpu().numpy(), ref.encode(col, starts=starts))
    d = np.tile(np.array([1, 4], np.uint64), 20_000)
    alternating = np.concatenate([[np.uint64(7)], np.uint64(7) + np.cumsum(d)]).astype(np.uint64)
    check(torch, codec, ref, alternating, "second-order deltas all 3", start_positions=True)
    check(torch, codec, ref, alternating, "second-order deltas all 3, tau 0, cap 3000",
          start_positions=True, tau=0.0, max_len=3000)
    wide = rng.integers(0, 2**64 - 1, 20_000, dtype=np.uint64, endpoint=True)
    wide[::3] = rng.integers(0, 16, len(wide[::3]), dtype=np.uint64)
    check(torch, codec, ref, wide, "65-bit differences", start_positions=True)
    for m in (1, 2, 3, 4, 5, 63, 64, 65, 127, 129):
        check(torch, codec, ref, W.constant_runs(m, 84 + m), f"n={m}", start_positions=True)
    big = 2 * (1 << 20) + 70_001
    check(torch, codec, ref, W.constant_runs(big, 85), "constant runs, 3 segments",
          start_positions=True)
    check(torch, codec, ref, W.piecewise_linear(big, 86, segments=300), "polyline, 3 segments",
          start_positions=True, tau=0.03)


def test_partition_params_are_checked(torch, codec):
    col = torch.from_numpy(W.linear_noise(1000, 87)).cuda()
    out = np.zeros(1001, dtype=np.uint64)
    for sp, res in ((2, 0), (-1, 0), (0, 1)):
        params = P.PartitionParams(0.1, 320, 1 << 20, 0, sp, res)
        st, _ = P.leco_partition(codec.ctx, col, 1000, P.LECO_U64, params, out)
        assert st == P.LECO_EINVAL
