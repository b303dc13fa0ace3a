"""The encoder that allocates nothing (leco_encode_noalloc) against
leco_encode_async: the same blob bytes and size on two calls in a row, the
second with a smaller input (the shared fixed scratch keeps the first
call's contents), for fixed and variable partitions and every regressor,
and a clear LECO_ENOSPC, before anything is enqueued, for a call whose
scratch would not fit the fixed array."""
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


def encode_both(torch, codec, col, **part_kw):
    """(async blob, no-alloc blob) of one column under one partitioning."""
    d = torch.from_numpy(np.ascontiguousarray(col)).cuda()
    dt = P.LECO_U32 if col.dtype == np.uint32 else P.LECO_U64
    part, keep = P.make_partitioning(**part_kw)
    cap = P.leco_max_blob_bytes(len(col), dt, part)
    out = []
    for fn in (P.leco_encode_async, P.leco_encode_noalloc):
        buf = torch.full((cap,), 0xA5, dtype=torch.uint8, device="cuda")
        size = torch.zeros(1, dtype=torch.uint64, device="cuda")
        codec.check(fn.__name__, fn(codec.ctx, d, len(col), dt, part, buf, cap, size))
        codec.sync()
        nbytes = int(size.cpu().numpy().view(np.uint64)[0])
        out.append(buf[:nbytes].cpu().numpy())
    del keep
    return out


@pytest.mark.parametrize("regressor", ["ls", "minimax", "poly"])
def test_noalloc_equals_async_twice(torch, codec, ref, regressor):
    """A large call, then a smaller one on the same fixed scratch: both equal
    the allocating encoder's blobs (and the oracle's)."""
    big = W.lognormal_keys(3_000_000, 201)
    small = W.linear_noise(70_001, 202, np.uint32)
    L = 1000 if regressor == "poly" else 4096
    for name, col in (("big", big), ("small", small)):
        log(f"[noalloc] {regressor} {name}: n={len(col)} fixed L={L}")
        a, b = encode_both(torch, codec, col, fixed_len=L, regressor=regressor)
        assert np.array_equal(a, b), f"{regressor} {name}: blobs differ"
        assert np.array_equal(b, ref.encode(col, fixed_len=L, regressor=regressor))


def test_noalloc_variable_partitions_twice(torch, codec, ref):
    col = W.constant_runs(400_000, 203)
    starts = ref.partition_greedy(col, tau=0.03)
    col2 = W.sorted_normal(50_000, 204)
    starts2 = ref.partition_greedy(col2, tau=0.03)
    for name, c, s in (("runs", col, starts), ("sorted normal", col2, starts2)):
        log(f"[noalloc] variable {name}: n={len(c)} m={len(s) - 1}")
        a, b = encode_both(torch, codec, c, starts=s)
        assert np.array_equal(a, b), f"{name}: blobs differ"
        assert np.array_equal(b, ref.encode(c, starts=s))


def test_noalloc_rejects_scratch_beyond_the_array(torch, codec):
    """Partitions of one value: about 56 bytes of scratch each, so 2^20
    partitions need more than the 32 MiB array: LECO_ENOSPC, and the
    context stays usable."""
    n = 1 << 20
    col = torch.arange(n, dtype=torch.int64, device="cuda")
    part, _ = P.make_partitioning(fixed_len=1)
    cap = P.leco_max_blob_bytes(n, P.LECO_U64, part)
    buf = torch.empty(cap, dtype=torch.uint8, device="cuda")
    size = torch.zeros(1, dtype=torch.uint64, device="cuda")
    log("[noalloc] 2^20 partitions: expect ENOSPC")
    st = P.leco_encode_noalloc(codec.ctx, col, n, P.LECO_U64, part, buf, cap, size)
    assert st == P.LECO_ENOSPC
    assert "scratch" in P.leco_last_error(codec.ctx)
    a, b = encode_both(torch, codec, W.linear_noise(10_000, 205), fixed_len=1024)
    assert np.array_equal(a, b)
