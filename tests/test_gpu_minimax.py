"""GPU parity of the minimax regressor (section 3.1's fixed-width
objective): blobs encoded on the GPU with the minimax regressor, through the
C ABI, against the oracle's bytes on the same seeded inputs, for fixed and
variable partitions, partitions spanning several hull tiles, and batches."""
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


def dev(torch, a: np.ndarray):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def same_blob(torch, codec, ref, col, name, fixed_len=0, starts=None, force_constant=False):
    log(f"[minimax] {name}: n={len(col)} dtype={col.dtype} L={fixed_len} "
        f"m={'-' if starts is None else len(starts) - 1}")
    expect = ref.encode(col, fixed_len=fixed_len, starts=starts, force_constant=force_constant,
                        regressor="minimax")
    blob = codec.encode(dev(torch, col), fixed_len=fixed_len, starts=starts,
                        force_constant=force_constant, regressor="minimax")
    got = blob.cpu().numpy()
    assert len(got) == len(expect), f"{name}: size {len(got)} != {len(expect)}"
    if not np.array_equal(got, expect):
        bad = np.flatnonzero(got != expect)
        raise AssertionError(f"{name}: {len(bad)} bytes differ, first at {bad[0]}")
    assert np.array_equal(codec.decode_all(blob).cpu().numpy(), col), f"{name}: decode_all"
    return len(got)


def convex(n, sign=1):
    t = np.arange(n, dtype=np.uint64)
    return t * t if sign > 0 else np.uint64(1 << 50) - t * t


def spiky(n, seed):
    rng = np.random.default_rng(seed)
    v = 1000 + 9 * np.arange(n, dtype=np.uint64) + rng.integers(0, 16, n).astype(np.uint64)
    idx = rng.integers(0, n, n // 300 + 1)
    v[idx] += rng.integers(0, 1 << 12, len(idx)).astype(np.uint64)
    return v


def steep_line(n, L, span, seed):
    """A noisy line whose partitions of L values each span about `span`
    (offsets from 2^61, noise below 2^20)."""
    rng = np.random.default_rng(seed)
    slope = np.uint64(span // (L - 1))
    t = np.arange(n, dtype=np.uint64)
    return np.uint64(1 << 61) + t * slope + rng.integers(0, 1 << 20, n).astype(np.uint64)


def periodic_bowl(n, L, shift):
    """(t mod L)^2 << shift above 2^62: every point of a partition is a
    lower-hull vertex, the range (L-1)^2 << shift."""
    t = np.arange(n, dtype=np.uint64) % np.uint64(L)
    return np.uint64(1 << 62) + ((t * t) << np.uint64(shift))


FIXED = [
    # hull tests in binary64 below a range of 2^40, in 128-bit integers above
    ("line_below_2_40_L1024", lambda: steep_line(100_000, 1024, (1 << 40) - (1 << 21), 40), 1024),
    ("line_above_2_40_L1024", lambda: steep_line(100_000, 1024, (1 << 40) + (1 << 21), 41), 1024),
    ("line_below_2_40_L4096", lambda: steep_line(100_000, 4096, (1 << 40) - (1 << 21), 42), 4096),
    ("bowl_below_2_40_L4096", lambda: periodic_bowl(40_000, 4096, 16), 4096),
    ("bowl_2_41_L4096", lambda: periodic_bowl(40_000, 4096, 17), 4096),
    ("bowl_L1024", lambda: periodic_bowl(40_000, 1024, 20), 1024),
    # every point collinear (hulls of two vertices after the ties), and
    # collinear runs meeting at corners
    ("exact_line", lambda: np.uint64(7) + np.arange(60_000, dtype=np.uint64) * np.uint64(3), 1024),
    ("exact_sawtooth", lambda: (np.arange(60_000, dtype=np.uint64) % np.uint64(37)) * np.uint64(5), 1000),
    ("exact_sawtooth_4096", lambda: (np.arange(60_000, dtype=np.uint64) % np.uint64(301)) * np.uint64(9), 4096),
    ("linear_noise", lambda: W.linear_noise(200_000, 1), 1024),
    ("lognormal_keys_u64", lambda: W.lognormal_keys(300_000, 2), 4096),
    ("lognormal_keys_u32", lambda: W.lognormal_keys(300_000, 3).astype(np.uint32), 4096),
    ("piecewise_u32", lambda: W.piecewise_linear(250_000, 32, segments=300).astype(np.uint32), 1000),
    ("constant_runs", lambda: W.constant_runs(120_000, 33), 777),
    ("convex", lambda: convex(50_000), 4096),
    ("concave", lambda: convex(30_000, -1), 2048),
    # every point a lower-hull vertex: the merge rounds' tangent searches
    # run over hulls of hundreds of vertices
    ("convex_1024", lambda: convex(60_000), 1024),
    ("rounded_root", lambda: np.floor(np.sqrt(np.arange(60_000.0)) * 1e6).astype(np.uint64), 1024),
    ("decreasing", lambda: (np.uint64(1 << 40) - W.lognormal_keys(100_000, 5)), 512),
    ("spiky", lambda: spiky(100_000, 6), 1024),
    ("uniform_wide", lambda: np.random.default_rng(7).integers(0, 1 << 60, 40_000, dtype=np.uint64), 300),
    ("range_2_61", lambda: np.random.default_rng(8).integers(0, 1 << 63, 20_000, dtype=np.uint64), 1024),
    ("tiny_partitions", lambda: W.linear_noise(5_000, 9), 3),
    ("pairs", lambda: W.linear_noise(4_001, 10), 2),
    ("singletons", lambda: W.linear_noise(1_000, 11), 1),
]


@pytest.mark.parametrize("name,make,L", FIXED, ids=[f[0] for f in FIXED])
def test_fixed_partitions_match_oracle(torch, codec, ref, name, make, L):
    col = make()
    size = same_blob(torch, codec, ref, col, name, fixed_len=L)
    # never larger than the least-squares blob
    assert size <= len(ref.encode(col, fixed_len=L))


def test_forced_constant_ignores_the_regressor(torch, codec, ref):
    col = W.linear_noise(30_000, 12)
    same_blob(torch, codec, ref, col, "forced", fixed_len=1024, force_constant=True)
    assert np.array_equal(ref.encode(col, fixed_len=1024, force_constant=True, regressor="minimax"),
                          ref.encode(col, fixed_len=1024, force_constant=True))


def test_partitions_spanning_several_hull_tiles(torch, codec, ref):
    """Variable partitions of 1 .. 2^20 values, several longer than one
    4096-point hull tile, on data whose hulls are short (noise) and long
    (a convex run, every point a lower-hull vertex)."""
    n = (1 << 20) + 300_000
    rng = np.random.default_rng(13)
    noise = W.linear_noise(n, 14)
    lens = [1, 2, 3, 4095, 4096, 4097, 9_000, 70_001, 1 << 20]
    starts = np.concatenate([[0], np.cumsum(lens)])
    rest = n - int(starts[-1])
    while rest > 0:
        k = int(min(rest, rng.integers(1, 30_000)))
        starts = np.append(starts, starts[-1] + k)
        rest -= k
    starts = starts.astype(np.uint64)
    same_blob(torch, codec, ref, noise, "variable_noise", starts=starts)
    bowl = convex(n)
    same_blob(torch, codec, ref, bowl, "variable_convex", starts=starts)


def test_fixed_partitions_longer_than_a_tile(torch, codec, ref):
    col = W.lognormal_keys((1 << 20) + 50_000, 15)
    same_blob(torch, codec, ref, col, "fixed_2_20", fixed_len=1 << 20)
    same_blob(torch, codec, ref, col[:200_000], "fixed_10000", fixed_len=10_000)


def test_batch_mixes_regressors(torch, codec, ref):
    """A batch of jobs with both regressors, partitions of 1024 (one
    wavefront each) and 8192 (two hull tiles): every blob equals the
    single-column encode and the oracle's."""
    specs = [(W.linear_noise(50_000, 20), 1024, 1), (W.linear_noise(40_000, 21), 1024, 0),
             (W.lognormal_keys(60_000, 22), 8192, 1), (spiky(30_000, 23).astype(np.uint32), 8192, 1),
             (convex(20_000), 8192, 0), (np.zeros(0, dtype=np.uint64), 1024, 1)]
    jobs, bufs, sizes, cols = [], [], [], []
    for col, L, reg in specs:
        d = dev(torch, col) if len(col) else torch.zeros(1, dtype=torch.uint64, device="cuda")
        dt = P.LECO_U32 if col.dtype == np.uint32 else P.LECO_U64
        part, _ = P.make_partitioning(fixed_len=L)
        cap = P.leco_max_blob_bytes(len(col), dt, part)
        buf = torch.zeros(cap, dtype=torch.uint8, device="cuda")
        size = torch.zeros(1, dtype=torch.uint64, device="cuda")
        job = P.EncodeJob(d.data_ptr() if len(col) else 0, len(col), dt, 0, L, buf.data_ptr(), cap,
                          size.data_ptr())
        job.regressor = reg
        jobs.append(job)
        bufs.append(buf)
        sizes.append(size)
        cols.append(d)
    log("[minimax] batch of 6 jobs")
    codec.check("leco_encode_batch", P.leco_encode_batch(codec.ctx, jobs))
    codec.sync()
    for (col, L, reg), buf, size in zip(specs, bufs, sizes):
        name = "minimax" if reg else "ls"
        got = buf[: int(size.item())].cpu().numpy()
        expect = ref.encode(col, fixed_len=L, regressor=name)
        assert np.array_equal(got, expect), f"batch job L={L} {name}"


def test_unknown_regressor_is_rejected(torch, codec):
    col = dev(torch, W.linear_noise(1000, 24))
    part, _ = P.make_partitioning(fixed_len=100)
    part.regressor = 3
    cap = 1 << 16
    buf = torch.zeros(cap, dtype=torch.uint8, device="cuda")
    st, _ = P.leco_encode(codec.ctx, col, 1000, P.LECO_U64, part, buf, cap, None)
    assert st == P.LECO_EINVAL
    with pytest.raises(ValueError):
        codec.encode(col, fixed_len=100, regressor="cubic")
