"""The one-pass encoders (fit, word offset by decoupled look-back, record
and packing in one kernel) against the oracle's bytes.  By default a context
takes them for launches of at most two workgroups per CU; the contexts under
test force them on (LECO_ENCODE_FUSED=1 for a workgroup per partition of
2049..4096 values, LECO_ENCODE_FUSED_WAVE=1 for a wavefront per partition
of at most 1024) or off (both 0, the two-pass encoder at small sizes).
Cases: both widths, ragged last partitions, the line, constant and FOR
models, residuals beyond 32 bits, variable partitions, and batches of many
columns (the look-back stops at each column's first partition)."""
from __future__ import annotations

import os

import numpy as np
import pytest

import paper_2306_15374_amd as P
from paper_2306_15374_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as T
    if not T.cuda.is_available():
        pytest.skip("no GPU")
    return T


@pytest.fixture(scope="module")
def codec(torch):
    old = os.environ.get("LECO_ENCODE_FUSED")
    os.environ["LECO_ENCODE_FUSED"] = "1"  # read when the context is created
    try:
        c = P.Codec(0)
    finally:
        if old is None:
            del os.environ["LECO_ENCODE_FUSED"]
        else:
            os.environ["LECO_ENCODE_FUSED"] = old
    yield c
    c.close()


def check(torch, codec, ref, col, name, **kw):
    print(f"[fused] {name}: n={len(col)} dtype={col.dtype} {sorted(kw)}", flush=True)
    expect = ref.encode(col, **kw)
    blob = codec.encode(torch.from_numpy(np.ascontiguousarray(col)).cuda(), **kw)
    got = blob.cpu().numpy()
    assert len(got) == len(expect), f"{name}: {len(got)} bytes != {len(expect)}"
    if not np.array_equal(got, expect):
        bad = np.flatnonzero(got != expect)
        raise AssertionError(f"{name}: {len(bad)} bytes differ, first at {bad[0]}")
    assert np.array_equal(codec.decode_all(blob).cpu().numpy(), col), f"{name}: round trip"


def test_fixed_lengths_and_models(torch, codec, ref):
    rng = np.random.default_rng(5)
    check(torch, codec, ref, W.lognormal_keys(300_000, 21), "sorted keys u64 L4096", fixed_len=4096)
    check(torch, codec, ref, W.lognormal_keys(250_001, 22, np.uint32), "keys u32 L3000 ragged",
          fixed_len=3000)
    check(torch, codec, ref, W.linear_noise(200_000, 23), "noise u64 L2049", fixed_len=2049)
    check(torch, codec, ref, np.full(50_000, 2**63 + 7, np.uint64), "constant (b=0) L4096",
          fixed_len=4096)
    check(torch, codec, ref, W.lognormal_keys(60_000, 24), "force constant L4096", fixed_len=4096,
          force_constant=True)
    wide = rng.integers(0, 2**40, 40_000, dtype=np.uint64)
    check(torch, codec, ref, wide, "40-bit noise (128-bit sums) L4096", fixed_len=4096)
    extreme = np.array([2**64 - 1, 0] * 20_000, np.uint64)
    check(torch, codec, ref, extreme, "wrap extremes (FOR) L2500", fixed_len=2500)
    steep = (np.arange(30_000, dtype=np.uint64) * np.uint64(2**40)).astype(np.uint64)
    check(torch, codec, ref, steep + rng.integers(0, 2**35, 30_000, dtype=np.uint64),
          "steep line, 64-bit predictions L4096", fixed_len=4096)
    check(torch, codec, ref, W.lognormal_keys(4096, 25), "one partition", fixed_len=4096)


def test_variable_partitions(torch, codec, ref):
    rng = np.random.default_rng(6)
    n = 120_000
    s = [0]
    while s[-1] < n:
        s.append(min(n, s[-1] + int(rng.choice([1, 2, 7, 300, 2049, 3000, 4096]))))
    starts = np.array(s, dtype=np.uint64)
    check(torch, codec, ref, W.piecewise_linear(n, 26, segments=40), "polyline u32 variable",
          starts=starts)
    check(torch, codec, ref, W.lognormal_keys(n, 27), "keys u64 variable", starts=starts)


def test_batch_of_columns(torch, codec, ref):
    specs = W.batched_columns(40, 9, lo=0, hi=200_000, median=15_000, sigma=1.5)
    specs[0]["n"] = 0
    specs[1]["n"] = 1
    specs[2]["n"] = 4097
    for i, s in enumerate(specs):
        s["fixed_len"] = [2049, 3000, 4096][i % 3]
    cols = [W.make_column_device(s) for s in specs]
    jobs, blobs, sizes = [], [], torch.zeros(len(specs), dtype=torch.uint64, device="cuda")
    for i, (s, c) in enumerate(zip(specs, cols)):
        dt = P.LECO_U32 if s["dtype"] == np.uint32 else P.LECO_U64
        part, _ = P.make_partitioning(fixed_len=s["fixed_len"])
        cap = P.leco_max_blob_bytes(s["n"], dt, part)
        buf = torch.empty(cap, dtype=torch.uint8, device="cuda")
        blobs.append(buf)
        jobs.append(P.EncodeJob(c.data_ptr() if s["n"] else 0, s["n"], dt, 0, s["fixed_len"],
                                buf.data_ptr(), cap, sizes.data_ptr() + 8 * i))
    print(f"[fused] batch of {len(specs)} columns", flush=True)
    codec.check("leco_encode_batch", P.leco_encode_batch(codec.ctx, jobs))
    codec.sync()
    sz = sizes.cpu().numpy().view(np.uint64)
    for i, (s, c) in enumerate(zip(specs, cols)):
        host = c.cpu().numpy().view(np.uint32 if s["dtype"] == np.uint32 else np.uint64)
        expect = ref.encode(host, fixed_len=s["fixed_len"])
        assert int(sz[i]) == len(expect), f"column {i}: size"
        assert np.array_equal(blobs[i][: int(sz[i])].cpu().numpy(), expect), f"column {i}: bytes"


def test_too_small_capacity_is_reported(torch, codec, ref):
    """A blob 16 bytes short: no write beyond it, ENOSPC with the size needed."""
    host = W.linear_noise(50_000, 28)
    need = len(ref.encode(host, fixed_len=4096))
    part, _ = P.make_partitioning(fixed_len=4096)
    small = torch.full((need,), 0xAB, dtype=torch.uint8, device="cuda")
    st, size = P.leco_encode(codec.ctx, torch.from_numpy(host).cuda(), len(host), P.LECO_U64,
                             part, small, need - 16)
    assert st == P.LECO_ENOSPC and size == need
    assert P.leco_sync(codec.ctx) == P.LECO_OK
    assert bool((small[need - 16:] == 0xAB).all()), "wrote past the capacity"


@pytest.fixture(scope="module")
def wave_codec(torch):
    """A context whose one-pass encoder takes one wavefront per partition
    (LECO_ENCODE_FUSED_WAVE=1: launches whose partitions hold at most 1024
    values)."""
    old = os.environ.get("LECO_ENCODE_FUSED_WAVE")
    os.environ["LECO_ENCODE_FUSED_WAVE"] = "1"
    try:
        c = P.Codec(0)
    finally:
        if old is None:
            del os.environ["LECO_ENCODE_FUSED_WAVE"]
        else:
            os.environ["LECO_ENCODE_FUSED_WAVE"] = old
    yield c
    c.close()


def test_wave_fixed_lengths_and_models(torch, wave_codec, ref):
    rng = np.random.default_rng(15)
    c = wave_codec
    check(torch, c, ref, W.linear_noise(300_000, 31), "noise u64 L1024", fixed_len=1024)
    check(torch, c, ref, W.lognormal_keys(250_001, 32, np.uint32), "keys u32 L1000 ragged",
          fixed_len=1000)
    check(torch, c, ref, W.lognormal_keys(20_000, 33), "keys u64 L64", fixed_len=64)
    check(torch, c, ref, W.lognormal_keys(3_001, 34), "L=1", fixed_len=1)
    check(torch, c, ref, np.full(50_000, 2**63 + 7, np.uint64), "constant (b=0) L1024",
          fixed_len=1024)
    check(torch, c, ref, W.lognormal_keys(60_000, 35), "force constant L1024", fixed_len=1024,
          force_constant=True)
    check(torch, c, ref, rng.integers(0, 2**64 - 1, 30_000, dtype=np.uint64, endpoint=True),
          "64-bit noise (b=64) L777", fixed_len=777)
    check(torch, c, ref, np.array([2**64 - 1, 0] * 20_000, np.uint64), "wrap extremes L100",
          fixed_len=100)


def test_wave_variable_partitions_and_batch(torch, wave_codec, ref):
    rng = np.random.default_rng(16)
    n = 120_000
    s = [0]
    while s[-1] < n:
        s.append(min(n, s[-1] + int(rng.choice([1, 2, 7, 63, 64, 65, 300, 1000, 1024]))))
    starts = np.array(s, dtype=np.uint64)
    check(torch, wave_codec, ref, W.piecewise_linear(n, 36, segments=40), "polyline u32 variable",
          starts=starts)
    specs = W.batched_columns(40, 17, lo=0, hi=200_000, median=15_000, sigma=1.5)
    specs[0]["n"] = 0
    specs[1]["n"] = 1
    specs[2]["n"] = 1025
    for i, sp in enumerate(specs):
        sp["fixed_len"] = [100, 1000, 1024][i % 3]
    cols = [W.make_column_device(sp) for sp in specs]
    jobs, blobs, sizes = [], [], torch.zeros(len(specs), dtype=torch.uint64, device="cuda")
    for i, (sp, col) in enumerate(zip(specs, cols)):
        dt = P.LECO_U32 if sp["dtype"] == np.uint32 else P.LECO_U64
        part, _ = P.make_partitioning(fixed_len=sp["fixed_len"])
        cap = P.leco_max_blob_bytes(sp["n"], dt, part)
        buf = torch.empty(cap, dtype=torch.uint8, device="cuda")
        blobs.append(buf)
        jobs.append(P.EncodeJob(col.data_ptr() if sp["n"] else 0, sp["n"], dt, 0, sp["fixed_len"],
                                buf.data_ptr(), cap, sizes.data_ptr() + 8 * i))
    print(f"[fused wave] batch of {len(specs)} columns", flush=True)
    wave_codec.check("leco_encode_batch", P.leco_encode_batch(wave_codec.ctx, jobs))
    wave_codec.sync()
    sz = sizes.cpu().numpy().view(np.uint64)
    for i, (sp, col) in enumerate(zip(specs, cols)):
        host = col.cpu().numpy().view(np.uint32 if sp["dtype"] == np.uint32 else np.uint64)
        expect = ref.encode(host, fixed_len=sp["fixed_len"])
        assert int(sz[i]) == len(expect), f"column {i}: size"
        assert np.array_equal(blobs[i][: int(sz[i])].cpu().numpy(), expect), f"column {i}: bytes"


@pytest.fixture(scope="module")
def two_pass_codec(torch):
    """A context with both one-pass encoders off."""
    keys = ("LECO_ENCODE_FUSED", "LECO_ENCODE_FUSED_WAVE")
    old = {k: os.environ.get(k) for k in keys}
    os.environ.update({k: "0" for k in keys})
    try:
        c = P.Codec(0)
    finally:
        for k, v in old.items():
            if v is None:
                del os.environ[k]
            else:
                os.environ[k] = v
    yield c
    c.close()


def test_two_pass_small_launches(torch, two_pass_codec, ref):
    c = two_pass_codec
    check(torch, c, ref, W.lognormal_keys(100_001, 41), "keys u64 L1024 (wavefront fit)",
          fixed_len=1024)
    check(torch, c, ref, W.lognormal_keys(100_000, 42, np.uint32), "keys u32 L2048 (32 per lane)",
          fixed_len=2048)
    check(torch, c, ref, W.linear_noise(100_000, 43), "noise u64 L4096", fixed_len=4096)
    check(torch, c, ref, W.linear_noise(100_000, 44), "noise u64 L5000", fixed_len=5000)
    rng = np.random.default_rng(45)
    n = 80_000
    s = [0]
    while s[-1] < n:
        s.append(min(n, s[-1] + int(rng.choice([1, 5, 64, 1000, 3000, 4096, 9000]))))
    check(torch, c, ref, W.piecewise_linear(n, 46, segments=20), "polyline u32 variable",
          starts=np.array(s, dtype=np.uint64))


def test_default_switches_at_two_workgroups_per_cu(torch, ref):
    """A default context takes the one-pass encoder up to two workgroups per
    CU and the two passes above: columns on both sides of the switch, for
    the wavefront kernel (partitions of 1024, four per workgroup) and the
    workgroup kernel (partitions of 4096), give the oracle's bytes."""
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    c = P.Codec(0)
    try:
        for L, per_wg in ((1024, 4), (4096, 1)):
            limit = 2 * cus * per_wg  # partitions at the switch
            for m in (limit, limit + 1):
                col = W.lognormal_keys(m * L - 7, 50 + m % 7)  # ragged last partition
                check(torch, c, ref, col, f"default L{L} m={m}", fixed_len=L)
    finally:
        c.close()
