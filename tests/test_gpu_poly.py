"""GPU parity of the polynomial regressor (degree 2 and 3 least squares in
the Gram basis): blobs encoded on the GPU through the C ABI against the
oracle's bytes, every decoder on such blobs against the oracle, batches
mixing regressors, and the paths that refuse polynomial blobs."""
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


def check(torch, codec, ref, col, name, fixed_len=0, starts=None, force_constant=False):
    log(f"[poly] {name}: n={len(col)} dtype={col.dtype} L={fixed_len} "
        f"m={'-' if starts is None else len(starts) - 1}")
    expect = ref.encode(col, fixed_len=fixed_len, starts=starts, force_constant=force_constant,
                        regressor="poly")
    blob = codec.encode(dev(torch, col), fixed_len=fixed_len, starts=starts,
                        force_constant=force_constant, regressor="poly")
    got = blob.cpu().numpy()
    assert len(got) == len(expect), f"{name}: size {len(got)} != {len(expect)}"
    if not np.array_equal(got, expect):
        bad = np.flatnonzero(got != expect)
        raise AssertionError(f"{name}: {len(bad)} bytes differ, first at {bad[0]}")
    assert codec.validate(blob) == P.LECO_OK
    n = len(col)
    assert np.array_equal(codec.decode_all(blob).cpu().numpy(), col), f"{name}: decode_all"
    assert np.array_equal(codec.decode_all(dev(torch, expect)).cpu().numpy(), col)
    if n:
        rng = np.random.default_rng(n)
        pos = rng.integers(0, n, size=3000, dtype=np.uint64)
        pos[:2] = [0, n - 1]
        ra = codec.random_access(blob, dev(torch, pos)).cpu().numpy()
        assert np.array_equal(ra, col[pos.astype(np.int64)]), f"{name}: random_access"
        b = int(rng.integers(0, n))
        e = int(min(n, b + rng.integers(1, 20_000)))
        rg = codec.decode_range(blob, b, e).cpu().numpy()
        assert np.array_equal(rg, col[b:e]), f"{name}: decode_range"
        lo = int(col.min()) + (int(col.max()) - int(col.min())) // 4
        hi = lo + (int(col.max()) - int(col.min())) // 2 + 1
        assert codec.filter_sum(blob, lo, hi) == ref.filter_sum(expect, lo, hi), f"{name}: filter"
    return len(got)


def wide(n, seed):
    return np.random.default_rng(seed).integers(0, 1 << 52, n, dtype=np.uint64)


def big_cubic(n, seed, L):
    """Cubic pieces of amplitude near 2^49.6 over an offset of 2^62, plus
    small noise: ranges just below the 2^50 limit of the polynomial fit, so
    its integer sums take their largest magnitudes."""
    rng = np.random.default_rng(seed)
    t = (np.arange(n) % L) / L
    v = np.floor((2.0 ** 49) * (t ** 3 + 0.5 * t)).astype(np.uint64)
    return v + rng.integers(0, 1000, n, dtype=np.uint64) + np.uint64(1 << 62)


FIXED = [
    ("cosmos_u32", lambda: W.cosmos(300_000, 1), 1000),
    ("cosmos_4096", lambda: W.cosmos(100_000, 2), 4096),
    ("poly_blocks_u64", lambda: W.poly_blocks(300_000, 3), 2000),
    ("poly_blocks_u32", lambda: (W.poly_blocks(200_000, 4) - np.uint64(1 << 40)).astype(np.uint32), 777),
    ("linear_noise", lambda: W.linear_noise(200_000, 5), 1024),
    ("lognormal_keys", lambda: W.lognormal_keys(200_000, 6), 4096),
    ("constant_runs", lambda: W.constant_runs(100_000, 7), 512),
    ("longer_than_4096", lambda: W.cosmos(60_000, 8), 5000),
    ("range_2_50", lambda: wide(30_000, 9), 1000),
    ("range_below_2_50_wave", lambda: big_cubic(50_000, 16, 1000), 1000),
    ("range_below_2_50_block", lambda: big_cubic(50_000, 17, 4096), 4096),
    ("range_below_2_50_wave32", lambda: big_cubic(50_000, 18, 2048), 2048),
    ("cosmos_1025", lambda: W.cosmos(50_000, 19), 1025),
    ("cosmos_2049", lambda: W.cosmos(50_000, 25), 2049),
    ("tiny_3", lambda: W.cosmos(5_000, 10), 3),
    ("tiny_4", lambda: W.cosmos(5_001, 11), 4),
    ("pairs", lambda: W.cosmos(4_001, 12), 2),
]


@pytest.mark.parametrize("name,make,L", FIXED, ids=[f[0] for f in FIXED])
def test_fixed_partitions_match_oracle(torch, codec, ref, name, make, L):
    check(torch, codec, ref, make(), name, fixed_len=L)


def test_variable_partitions_match_oracle(torch, codec, ref):
    col = W.poly_blocks(400_000, 13)
    rng = np.random.default_rng(14)
    starts = [0]
    while starts[-1] < len(col):
        starts.append(min(len(col), starts[-1] + int(rng.choice([1, 2, 3, 4, 100, 4096, 4097, 9000]))))
    check(torch, codec, ref, col, "variable", starts=np.array(starts, dtype=np.uint64))


def test_forced_constant(torch, codec, ref):
    check(torch, codec, ref, W.cosmos(20_000, 15), "forced", fixed_len=1000, force_constant=True)


def test_batch_mixes_regressors(torch, codec, ref):
    specs = [(W.cosmos(50_000, 20), 1000, 2), (W.linear_noise(40_000, 21), 1024, 0),
             (W.poly_blocks(60_000, 22), 8192, 2), (W.lognormal_keys(30_000, 23), 4096, 1),
             (W.cosmos(20_000, 24), 512, 0), (np.zeros(0, dtype=np.uint64), 1024, 2)]
    jobs, bufs, sizes = [], [], []
    keep = []
    for col, L, reg in specs:
        d = dev(torch, col) if len(col) else torch.zeros(1, dtype=torch.uint64, device="cuda")
        keep.append(d)
        dt = P.LECO_U32 if col.dtype == np.uint32 else P.LECO_U64
        part, _ = P.make_partitioning(fixed_len=L, regressor=["ls", "minimax", "poly"][reg])
        cap = P.leco_max_blob_bytes(len(col), dt, part)
        buf = torch.zeros(cap, dtype=torch.uint8, device="cuda")
        size = torch.zeros(1, dtype=torch.uint64, device="cuda")
        job = P.EncodeJob(d.data_ptr() if len(col) else 0, len(col), dt, 0, L, buf.data_ptr(), cap,
                          size.data_ptr())
        job.regressor = reg
        jobs.append(job)
        bufs.append(buf)
        sizes.append(size)
    log("[poly] batch of 6 jobs")
    codec.check("leco_encode_batch", P.leco_encode_batch(codec.ctx, jobs))
    codec.sync()
    for (col, L, reg), buf, size in zip(specs, bufs, sizes):
        name = ["ls", "minimax", "poly"][reg]
        got = buf[: int(size.item())].cpu().numpy()
        assert np.array_equal(got, ref.encode(col, fixed_len=L, regressor=name)), f"L={L} {name}"


def test_batched_decode_and_filter_of_polynomial_blobs(torch, codec, ref):
    """One batch of polynomial and linear blobs: decoded values and fused
    filter sums equal the columns (polynomial tiles take the value-by-value
    path inside the same launch)."""
    cols = [W.cosmos(50_000, 40), W.poly_blocks(80_000, 41), W.linear_noise(30_000, 42),
            W.cosmos(7_777, 43)]
    regs = ["poly", "poly", "ls", "poly"]
    blobs, outs, sums, jobs = [], [], [], []
    for col, reg in zip(cols, regs):
        b = codec.encode(dev(torch, col), fixed_len=1000, regressor=reg)
        o = torch.zeros(len(col), dtype=torch.uint32 if col.dtype == np.uint32 else torch.uint64,
                        device="cuda")
        s3 = torch.zeros(3, dtype=torch.uint64, device="cuda")
        lo = int(col.min()) + (int(col.max()) - int(col.min())) // 3
        hi = lo + (int(col.max()) - int(col.min())) // 3
        jobs.append(P.DecodeJob(b.data_ptr(), b.numel(), len(col), o.data_ptr(), lo, hi, s3.data_ptr()))
        blobs.append(b)
        outs.append(o)
        sums.append((s3, lo, hi))
    handle = P.leco_batch_create(codec.ctx, jobs)
    try:
        for op in (P.LECO_BATCH_DECODE, P.LECO_BATCH_DECODE | P.LECO_BATCH_FILTER):
            for o in outs:
                o.zero_()
            assert P.leco_batch_run(handle, op) == P.LECO_OK
            codec.sync()
            for col, o in zip(cols, outs):
                assert np.array_equal(o.cpu().numpy(), col)
        for col, (s3, lo, hi) in zip(cols, sums):
            v = [int(x) for x in s3.cpu().numpy()]
            sel = col[(col >= lo) & (col < hi)].astype(object)
            assert ((v[1] << 64) | v[0], v[2]) == (int(sum(sel)), len(sel))
    finally:
        P.leco_batch_destroy(handle)


def test_validation_of_kind_bytes(torch, codec):
    col = W.cosmos(10_000, 31)
    ls = codec.encode(dev(torch, col), fixed_len=1000)
    bad = ls.clone()
    bad[64 + 25] = 1  # a polynomial kind in a blob without coefficients
    assert codec.validate(bad) == P.LECO_EFORMAT
    poly = codec.encode(dev(torch, col), fixed_len=1000, regressor="poly")
    assert codec.validate(poly) == P.LECO_OK
    bad = poly.clone()
    bad[64 + 25] = 2
    assert codec.validate(bad) == P.LECO_EFORMAT


def test_size_search_with_polynomials(torch, codec, ref):
    col = W.poly_blocks(500_000, 32)
    starts = W.sample_window_starts(len(col), 8_000, fraction=0.05, seed=33)
    d = dev(torch, col)
    for L in (3, 500, 4096, 8000):
        assert codec.fixed_cost(d, starts, 8_000, L, regressor="poly") == \
            ref.fixed_cost(col, starts, 8_000, L, regressor="poly")
    assert codec.size_search(d, starts, 8_000, regressor="poly") == \
        ref.size_search(col, starts, 8_000, regressor="poly")


@pytest.mark.parametrize("env", [{"LECO_ENCODE_WAVE32": "0"}, {"LECO_ENCODE_WAVE": "0"}])
def test_fit_kernel_choice_keeps_bytes(torch, ref, monkeypatch, env):
    """Partitions of 1025..2048 values fitted one per workgroup (wavefronts
    of 32 values per lane switched off) and of at most 1024 (wavefronts
    switched off): the same bytes as the oracle, least squares and
    polynomials."""
    for k, v in env.items():
        monkeypatch.setenv(k, v)
    c = P.Codec(0)
    try:
        for name, col, L in [("cosmos", W.cosmos(60_000, 26), 2000),
                             ("poly_blocks", W.poly_blocks(60_000, 27), 1000)]:
            for reg in ("ls", "poly"):
                log(f"[poly] {env} {name} L={L} {reg}")
                expect = ref.encode(col, fixed_len=L, regressor=reg)
                got = c.encode(dev(torch, col), fixed_len=L, regressor=reg).cpu().numpy()
                assert np.array_equal(got, expect), f"{env} {name} {reg}"
    finally:
        c.close()
