"""GPU parity: the HIP path, called through the C ABI, against the CPU oracle
on the same seeded inputs.  Bytes of every blob and every decoded value must
be identical (integer work: bit-exact)."""
from __future__ import annotations

import math
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


def host(t) -> np.ndarray:
    return t.cpu().numpy()


def random_partitioning(rng, n: int, max_len: int):
    s = [0]
    while s[-1] < n:
        s.append(min(n, s[-1] + int(rng.integers(1, max_len + 1))))
    return np.array(s, dtype=np.uint64)


def check_column(torch, codec, ref, col: np.ndarray, name: str, fixed_len: int = 0, starts=None,
                 force_constant: bool = False, ra: int = 2000, seed: int = 0):
    """Encode on both sides and compare bytes; decode every way and compare."""
    log(f"[parity] {name}: n={len(col)} dtype={col.dtype} L={fixed_len} "
        f"m={'-' if starts is None else len(starts) - 1}")
    rng = np.random.default_rng(seed)
    expect = ref.encode(col, fixed_len=fixed_len, starts=starts, force_constant=force_constant)
    d = dev(torch, col)
    blob = codec.encode(d, fixed_len=fixed_len, starts=starts, force_constant=force_constant)
    got = host(blob)
    assert len(got) == len(expect), f"{name}: size {len(got)} != {len(expect)}"
    if not np.array_equal(got, expect):
        bad = np.flatnonzero(got != expect)
        raise AssertionError(f"{name}: {len(bad)} bytes differ, first at {bad[0]}")
    assert codec.validate(blob) == P.LECO_OK
    n = len(col)
    out = codec.decode_all(blob)
    assert np.array_equal(host(out), col), f"{name}: decode_all"
    # decoding the oracle's blob gives the same
    out2 = codec.decode_all(dev(torch, expect))
    assert np.array_equal(host(out2), col)
    if n:
        pos = rng.integers(0, n, size=ra, dtype=np.uint64)
        pos[:3] = [0, n - 1, n // 2]
        r = codec.random_access(blob, dev(torch, pos))
        assert np.array_equal(host(r), ref.random_access(expect, pos)), f"{name}: random_access"
        for _ in range(4):
            b = int(rng.integers(0, n))
            e = int(rng.integers(b, n + 1))
            r = codec.decode_range(blob, b, e)
            assert np.array_equal(host(r), col[b:e]), f"{name}: decode_range {b}:{e}"
        lo, hi = sorted(int(x) for x in rng.choice(col, 2))
        assert codec.filter_sum(blob, lo, hi) == ref.filter_sum(expect, lo, hi), f"{name}: filter"
    return blob, expect


# ---- workload-shaped cases (scaled so the oracle finishes in seconds) ---------

def test_linear_noise_full_size(torch, codec, ref):
    col = W.linear_noise(W.C1_N, W.C1_SEED)
    blob, expect = check_column(torch, codec, ref, col, "linear_noise 1e6 L=1024",
                                fixed_len=W.C1_L, ra=10)
    pos = W.uniform_positions(W.C1_N, W.C1_RA, W.C1_RA_SEED)
    r = codec.random_access(blob, dev(torch, pos))
    assert np.array_equal(host(r), ref.random_access(expect, pos))
    assert np.array_equal(host(r), col[pos])


@pytest.mark.parametrize("dtype", [np.uint64, np.uint32])
def test_lognormal_keys_scaled(torch, codec, ref, dtype):
    col = W.lognormal_keys(2_000_000 + 123, W.C2_SEED, dtype)
    check_column(torch, codec, ref, col, f"lognormal_keys 2e6 {dtype.__name__}",
                 fixed_len=W.C2_L)


def test_linear_noise_u32_tail(torch, codec, ref):
    col = W.linear_noise(300_001, 5, np.uint32)
    check_column(torch, codec, ref, col, "linear_noise u32", fixed_len=1000)


@pytest.mark.parametrize("kind", ["sorted_normal", "piecewise_linear", "constant_runs"])
def test_mixed_distributions_variable_partitions(torch, codec, ref, kind):
    n = 200_000
    col = {"sorted_normal": lambda: W.sorted_normal(n, W.C3_SEEDS[0]),
           "piecewise_linear": lambda: W.piecewise_linear(n, W.C3_SEEDS[1], segments=50),
           "constant_runs": lambda: W.constant_runs(n, W.C3_SEEDS[2])}[kind]()
    starts = ref.partition_greedy(col, tau=0.1, sm_bits=320)
    check_column(torch, codec, ref, col, f"{kind} greedy", starts=starts)
    check_column(torch, codec, ref, col, f"{kind} fixed", fixed_len=2048)


# ---- edge cases ------------------------------------------------------------------

def test_edge_cases(torch, codec, ref):
    rng = np.random.default_rng(9)
    cases = [
        ("empty u64", np.zeros(0, np.uint64), dict(fixed_len=1024)),
        ("empty u32 var", np.zeros(0, np.uint32), dict(starts=[0])),
        ("single", np.array([12345], np.uint64), dict(fixed_len=4096)),
        ("L=1", W.lognormal_keys(3000, 4), dict(fixed_len=1)),
        ("full range u64 (b=64)", rng.integers(0, 2**64 - 1, 5000, np.uint64, endpoint=True),
         dict(fixed_len=512)),
        ("full range u32 (b=32)", rng.integers(0, 2**32 - 1, 5000, np.uint64,
                                               endpoint=True).astype(np.uint32), dict(fixed_len=300)),
        ("constant (b=0)", np.full(10_000, 2**63 + 7, np.uint64), dict(fixed_len=4096)),
        ("decreasing", (2**64 - 1 - np.arange(20_000, dtype=np.uint64) * np.uint64(1000) -
                        rng.integers(0, 50, 20_000, dtype=np.uint64)), dict(fixed_len=1024)),
        ("wrap extremes", np.array([2**64 - 1, 0] * 3000, np.uint64), dict(fixed_len=100)),
        ("huge ranges", np.sort(rng.integers(0, 2**64 - 1, 9000, np.uint64, endpoint=True)),
         dict(fixed_len=4096)),
        ("force constant", W.lognormal_keys(50_000, 6), dict(fixed_len=4096, force_constant=True)),
        ("var lengths 1..50", W.linear_noise(20_000, 7),
         dict(starts=random_partitioning(rng, 20_000, 50))),
        ("var long", W.lognormal_keys(70_000, 8),
         dict(starts=np.array([0, 1, 2, 30_000, 69_999, 70_000], np.uint64))),
        ("max partition", W.lognormal_keys((1 << 20) + 5, 3), dict(fixed_len=1 << 20)),
        ("L=4097 ragged", W.lognormal_keys(100_000, 10, np.uint32), dict(fixed_len=4097)),
        # one wavefront per partition with 32 values per lane (1025..2048)
        ("L=1025 u32", W.lognormal_keys(60_000, 11, np.uint32), dict(fixed_len=1025)),
        ("L=2048 full range", rng.integers(0, 2**64 - 1, 9000, np.uint64, endpoint=True),
         dict(fixed_len=2048)),
        ("L=2049", W.linear_noise(30_000, 12), dict(fixed_len=2049)),
    ]
    for name, col, kw in cases:
        check_column(torch, codec, ref, col, name, **kw)


def test_wide_residuals_across_chunks(torch, codec, ref):
    """Widths above 32 bits: the tile size picked from the blob's bits per
    value keeps each wavefront's words within one LDS slice."""
    rng = np.random.default_rng(12)
    t = np.arange(200_000, dtype=np.uint64)
    col = t * np.uint64(2**20) + rng.integers(0, 2**45, 200_000, dtype=np.uint64)
    check_column(torch, codec, ref, col, "b~45 L=65536", fixed_len=65536)
    check_column(torch, codec, ref, col, "b~45 L=4096", fixed_len=4096)


@pytest.mark.parametrize("tile_log2", [8, 14])
def test_fixed_tile_shapes(torch, ref, monkeypatch, tile_log2):
    """Tile size fixed through the environment instead of picked per blob.
    At 2^14 values per tile (4096 per wavefront) the 45-bit residuals and the
    ~14-bit residuals of sorted keys overflow the wavefront's LDS slice and go
    through the chunked path; at 2^8 a partition spans many wavefronts and
    tiles."""
    monkeypatch.setenv("LECO_TILE_LOG2", str(tile_log2))
    c = P.Codec(0)
    try:
        rng = np.random.default_rng(13)
        t = np.arange(150_000, dtype=np.uint64)
        wide = t * np.uint64(2**20) + rng.integers(0, 2**45, 150_000, dtype=np.uint64)
        check_column(torch, c, ref, wide, f"tile 2^{tile_log2} b~45", fixed_len=4096)
        mid = W.linear_noise(150_003, 14, np.uint32)
        check_column(torch, c, ref, mid, f"tile 2^{tile_log2} u32", fixed_len=1000)
        var = W.lognormal_keys(60_000, 15)
        check_column(torch, c, ref, var, f"tile 2^{tile_log2} variable",
                     starts=random_partitioning(rng, 60_000, 3000))
    finally:
        c.close()


# ---- short partitions: pieces decoded lane by lane across partition boundaries ----

def short_partition_cases(rng):
    """Columns whose partitions are short enough (tens to a few hundred values)
    for a wavefront to decode a run of them in full 64-value rounds."""
    n = 40_000
    t = np.arange(n, dtype=np.uint64)
    decreasing = (np.uint64(2**63) - t * np.uint64(977) - rng.integers(0, 300, n, dtype=np.uint64))
    wide = t * np.uint64(2**40) + rng.integers(0, 2**38, n, dtype=np.uint64)
    runs = W.constant_runs(n, 34)
    full32 = rng.integers(0, 2**32 - 1, 5000, np.uint64, endpoint=True).astype(np.uint32)
    mixed = np.concatenate([W.linear_noise(10_000, 35), np.sort(rng.integers(0, 2**62, 10_000,
                                                                            dtype=np.uint64)),
                            np.full(10_000, 42, np.uint64), decreasing[:10_000]])
    return [
        ("short decreasing u64 (negative slopes)", decreasing,
         dict(starts=random_partitioning(rng, n, 40))),
        ("short wide u64 (b~38, large predictions)", wide,
         dict(starts=random_partitioning(rng, n, 60))),
        ("short constant runs u32 (greedy)", runs, dict(starts=None)),
        ("L=7 full range u32 (b=32)", full32, dict(fixed_len=7)),
        ("L=200 linear noise u64", W.linear_noise(50_001, 36), dict(fixed_len=200)),
        ("L=33 linear noise u32", W.linear_noise(30_000, 37, np.uint32), dict(fixed_len=33)),
        ("short mixed generators u64", mixed, dict(starts=random_partitioning(rng, len(mixed), 300))),
    ]


def test_short_partitions(torch, codec, ref):
    rng = np.random.default_rng(33)
    for name, col, kw in short_partition_cases(rng):
        if "starts" in kw and kw["starts"] is None:
            kw = dict(starts=ref.partition_greedy(col, tau=0.1, sm_bits=320))
        check_column(torch, codec, ref, col, name, **kw)


@pytest.mark.parametrize("tile_log2", [8, 11, 14])
def test_short_partitions_tile_shapes(torch, ref, monkeypatch, tile_log2):
    """Wavefront shares of 64, 512 and 4096 values: pieces start inside a
    partition, end at the share's end, and span up to the bitmap's size."""
    monkeypatch.setenv("LECO_TILE_LOG2", str(tile_log2))
    c = P.Codec(0)
    try:
        rng = np.random.default_rng(34)
        for name, col, kw in short_partition_cases(rng)[:2] + short_partition_cases(rng)[4:5]:
            check_column(torch, c, ref, col, f"tile 2^{tile_log2} {name}", **kw)
    finally:
        c.close()


@pytest.mark.parametrize("env", [{"LECO_TILE_LOG2": "8"}, {"LECO_TILE_LOG2": "9"},
                                 {"LECO_TILE_LOG2": "11", "LECO_DECODE_BLOCKS_PER_CU": "1"}])
def test_variable_blob_tile_shapes(torch, ref, monkeypatch, env):
    """Variable-length blobs with short and long partitions at tiles of 256
    and 512 values, and with a persistent grid of one workgroup per CU that
    walks many tiles: decode_all, ranges and the filter sum."""
    for k, v in env.items():
        monkeypatch.setenv(k, v)
    c = P.Codec(0)
    try:
        rng = np.random.default_rng(35)
        n = 1_200_000
        runs = W.constant_runs(n, 36)
        check_column(torch, c, ref, runs, f"{env} constant runs greedy",
                     starts=ref.partition_greedy(runs, tau=0.1, sm_bits=320))
        noise = W.linear_noise(n, 37)
        check_column(torch, c, ref, noise, f"{env} linear noise 1..3000",
                     starts=random_partitioning(rng, n, 3000))
        check_column(torch, c, ref, noise[:400_000], f"{env} linear noise 1..20",
                     starts=random_partitioning(rng, 400_000, 20))
    finally:
        c.close()


# ---- slope arithmetic ------------------------------------------------------------

def test_device_slope_matches_host_rounding(torch, codec):
    """fl(N)/fl(D) on the GPU equals Python's correctly rounded int->float
    conversion followed by an IEEE division, over edge cases and 10^6
    random pairs in the ranges the fit produces (|N| < 2^121, D < 2^80)."""
    rng = np.random.default_rng(5)
    pairs = []
    edge_n = [0, 1, -1, 2**53 - 1, 2**53, 2**53 + 1, 2**53 + 2, 2**53 + 3, -(2**53 + 1),
              2**64 - 1, 2**64, 2**64 + 1, 2**65 + 2**12, 2**65 + 2**12 + 1, (1 << 120) - 1,
              -(1 << 120), (1 << 63) + (1 << 10), (1 << 63) + (1 << 10) + 1, (1 << 63) + (3 << 10),
              (2**54 + 1) << 60, ((2**53 + 1) << 66) + 1, -(((2**53 + 1) << 66))]
    edge_d = [1, 3, 12, 2**53 + 1, (1 << 79) + 12345, 2**64 + 1, 2**79 - 1]
    for a in edge_n:
        for b in edge_d:
            pairs.append((a, b))
    for _ in range(1_000_000 - len(pairs)):
        nb = int(rng.integers(1, 121))
        a = int(rng.integers(0, 2**63)) << max(0, nb - 63) | int(rng.integers(0, 2**63))
        a &= (1 << nb) - 1
        if rng.integers(0, 2):
            a = -a
        db = int(rng.integers(1, 80))
        b = (int(rng.integers(0, 2**63)) << max(0, db - 63) | int(rng.integers(1, 2**63)))
        b = (b & ((1 << db) - 1)) or 1
        pairs.append((a, b))
    k = len(pairs)
    arr = np.zeros((k, 4), dtype=np.uint64)
    for i, (a, b) in enumerate(pairs):
        ua = a % (1 << 128)
        arr[i] = [ua & (2**64 - 1), ua >> 64, b & (2**64 - 1), b >> 64]
    out = torch.empty(k, dtype=torch.float64, device="cuda")
    codec.check("leco_diag_slope", P.leco_diag_slope(codec.ctx, dev(torch, arr.reshape(-1)), k, out))
    codec.sync()
    got = host(out)
    expect = np.array([float(a) / float(b) for a, b in pairs])
    expect[expect == 0.0] = 0.0
    assert np.array_equal(got.view(np.uint64), expect.view(np.uint64))


# ---- error paths -----------------------------------------------------------------

def test_error_paths(torch, codec, ref):
    col = W.linear_noise(10_000, 3)
    blob = codec.encode(dev(torch, col), fixed_len=1000)
    # position >= n: flagged on the device, reported by the next sync
    pos = dev(torch, np.array([5, 10_000, 7], dtype=np.uint64))
    out = torch.empty(3, dtype=torch.uint64, device="cuda")
    assert P.leco_random_access(codec.ctx, blob, blob.numel(), pos, 3, out) == P.LECO_OK
    assert P.leco_sync(codec.ctx) == P.LECO_ERANGE
    assert P.leco_sync(codec.ctx) == P.LECO_OK  # flag cleared
    # range past the end
    out = torch.empty(10, dtype=torch.uint64, device="cuda")
    assert P.leco_decode_range(codec.ctx, blob, blob.numel(), 9_995, 10_005, out) == P.LECO_OK
    assert P.leco_sync(codec.ctx) == P.LECO_ERANGE
    assert P.leco_decode_range(codec.ctx, blob, blob.numel(), 10, 5, out) == P.LECO_ERANGE
    # output too small for decode_all
    assert P.leco_decode_all(codec.ctx, blob, blob.numel(), out, 10) == P.LECO_OK
    assert P.leco_sync(codec.ctx) == P.LECO_ENOSPC
    # corrupt magic and record width: kernels refuse, validation names it
    bad = blob.clone()
    bad[0] ^= 1
    big = torch.empty(10_000, dtype=torch.uint64, device="cuda")
    assert P.leco_decode_all(codec.ctx, bad, bad.numel(), big, 10_000) == P.LECO_OK
    assert P.leco_sync(codec.ctx) == P.LECO_EFORMAT
    assert codec.validate(bad) == P.LECO_EFORMAT
    bad = blob.clone()
    bad[64 + 24] = 65  # width of partition 0
    assert P.leco_decode_all(codec.ctx, bad, bad.numel(), big, 10_000) == P.LECO_OK
    assert P.leco_sync(codec.ctx) == P.LECO_EFORMAT
    assert codec.validate(bad) == P.LECO_EFORMAT
    # truncated blob
    assert P.leco_decode_all(codec.ctx, blob, blob.numel() - 16, big, 10_000) == P.LECO_OK
    assert P.leco_sync(codec.ctx) == P.LECO_EFORMAT
    # encode capacity too small: required size is returned
    need = len(ref.encode(col, fixed_len=1000))
    part, _ = P.make_partitioning(fixed_len=1000)
    small = torch.empty(need - 16, dtype=torch.uint8, device="cuda")
    st, size = P.leco_encode(codec.ctx, dev(torch, col), len(col), P.LECO_U64, part, small,
                             need - 16)
    assert st == P.LECO_ENOSPC and size == need
    assert P.leco_sync(codec.ctx) == P.LECO_OK
    # bad partitioning is rejected on the host
    part, keep = P.make_partitioning(starts=[0, 10, 10, 10_000])
    st, _ = P.leco_encode(codec.ctx, dev(torch, col), len(col), P.LECO_U64, part, small, need)
    assert st == P.LECO_EINVAL


def test_encode_async_matches_sync(torch, codec, ref):
    col = W.lognormal_keys(300_000, 13)
    part, _ = P.make_partitioning(fixed_len=4096)
    cap = P.leco_max_blob_bytes(len(col), P.LECO_U64, part)
    buf = torch.empty(cap, dtype=torch.uint8, device="cuda")
    size = torch.zeros(1, dtype=torch.uint64, device="cuda")
    assert P.leco_encode_async(codec.ctx, dev(torch, col), len(col), P.LECO_U64, part, buf, cap,
                               size) == P.LECO_OK
    codec.sync()
    s = int(host(size)[0])
    assert np.array_equal(host(buf[:s]), ref.encode(col, fixed_len=4096))


def test_short_partitions_one_thread_each(torch, codec, ref):
    """Launches whose partitions hold at most 32 values (more than 2,048 of
    them, so the two-pass encoder runs) are fitted one thread per
    partition: both widths, lengths 1..32 with ragged last partitions, the
    constant model forced, ranges at and beyond 2^61."""
    rng = np.random.default_rng(91)
    keys = W.lognormal_keys(120_001, 92)
    for L in (1, 2, 3, 17, 32):
        check_column(torch, codec, ref, keys, f"keys u64 L={L}", fixed_len=L, ra=200)
    check_column(torch, codec, ref, W.linear_noise(100_003, 93, np.uint32), "noise u32 L=31",
                 fixed_len=31, ra=200)
    check_column(torch, codec, ref, keys, "forced constant L=8", fixed_len=8, force_constant=True,
                 ra=200)
    wide = rng.integers(0, 2**64 - 1, 80_000, dtype=np.uint64, endpoint=True)
    check_column(torch, codec, ref, wide, "64-bit noise L=32", fixed_len=32, ra=200)
    edge = np.where(rng.random(80_000) < 0.5, np.uint64(0), np.uint64(2**61)).astype(np.uint64)
    check_column(torch, codec, ref, edge, "range exactly 2^61 L=16", fixed_len=16, ra=200)


def test_narrow_residual_boundaries(torch, codec, ref):
    """The register-held fits take residuals in 32 bits when the partition's
    range is below 2^30 and every |floor(theta1 t)| stays below 2^30: lines
    of slope 2^20 +- 1 per value over partitions of 1024 (|theta1| len on
    either side of 2^30, range just below it), rising and falling, ranges of
    exactly 2^30 - 1 and 2^30, both widths, the u64 ones offset by 2^40, at
    L 1024 (one wavefront per partition), 2000 (32 per lane) and 4096 (one
    workgroup)."""
    rng = np.random.default_rng(95)
    n = 40 * 4096 + 777
    for L in (1024, 2000, 4096):
        t = np.arange(n, dtype=np.uint64) % np.uint64(L)
        noise = rng.integers(0, 16, n).astype(np.uint64)
        cols = {}
        for slope in ((1 << 30) // L - 1, (1 << 30) // L + 1):
            s = np.uint64(slope)
            cols[f"rising slope {slope}"] = s * t + noise
            cols[f"falling slope {slope}"] = s * (np.uint64(L - 1) - t) + noise
        for r in ((1 << 30) - 1, 1 << 30):
            spike = (rng.random(n) < 0.01) | (t == np.uint64(L // 2))
            cols[f"range {r}"] = np.where(spike, np.uint64(r), noise).astype(np.uint64)
        for name, v in cols.items():
            if int(v.max()) < 2**32:
                check_column(torch, codec, ref, v.astype(np.uint32), f"u32 {name} L={L}",
                             fixed_len=L, ra=200)
            check_column(torch, codec, ref, v + np.uint64(1 << 40), f"u64 {name} L={L}",
                         fixed_len=L, ra=200)


def test_wide_range_sums_at_their_bounds(torch, codec, ref):
    """Partitions spanning just under 2^61 (the largest range a line is
    fitted to), with a trend so that the fit matters, at the longest
    partitions each wavefront fit holds (1024 and 2048 values) and at 4096:
    the wide-range sums at their largest magnitudes."""
    rng = np.random.default_rng(97)
    n = 24 * 4096 + 333
    top = (1 << 61) - 1
    for L in (1024, 2048, 4096):
        t = (np.arange(n) % L).astype(np.float64) / (L - 1)
        trend = (t * (top - (1 << 58))).astype(np.uint64)
        col = trend + rng.integers(0, 1 << 58, n, dtype=np.uint64)
        col[np.arange(n) % L == 0] = 0  # every partition spans close to 2^61
        assert int(col.max()) <= top
        check_column(torch, codec, ref, col, f"near 2^61 L={L}", fixed_len=L, ra=200)
