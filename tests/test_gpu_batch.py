"""Batched mode on the GPU: one encode launch and one decode launch over many
columns must give exactly the bytes and values of the single-column calls
and of the oracle, for every launch shape, eagerly and from a HIP graph."""
from __future__ import annotations

import sys

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
    c = P.Codec(0)
    yield c
    c.close()


def np_view(t, dtype):
    a = t.cpu().numpy()
    return a.view(np.uint32 if dtype == np.uint32 else np.uint64)


def small_specs(ncols=48, seed=7):
    """Columns shaped like the batched workload but small: lognormal lengths
    (with an empty, a single-value and a ragged column), mixed dtypes and
    generators."""
    specs = W.batched_columns(ncols, seed, lo=0, hi=300_000, median=20_000, sigma=1.5)
    specs[0]["n"] = 0
    specs[1]["n"] = 1
    specs[2]["n"] = 4097
    return specs


def encode_batch(torch, codec, specs, cols):
    jobs, blobs, sizes = [], [], torch.zeros(len(specs), dtype=torch.uint64, device="cuda")
    for i, (s, c) in enumerate(zip(specs, cols)):
        dt = P.LECO_U32 if s["dtype"] == np.uint32 else P.LECO_U64
        part, _ = P.make_partitioning(fixed_len=s["fixed_len"])
        cap = P.leco_max_blob_bytes(s["n"], dt, part)
        buf = torch.empty(cap, dtype=torch.uint8, device="cuda")
        blobs.append(buf)
        jobs.append(P.EncodeJob(c.data_ptr() if s["n"] else 0, s["n"], dt, 0, s["fixed_len"],
                                buf.data_ptr(), cap, sizes.data_ptr() + 8 * i))
    codec.check("leco_encode_batch", P.leco_encode_batch(codec.ctx, jobs))
    codec.sync()
    sz = sizes.cpu().numpy().view(np.uint64)
    return [b[: int(n)] for b, n in zip(blobs, sz)]


def test_batch_encode_matches_single_and_oracle(torch, codec, ref):
    specs = small_specs()
    cols = [W.make_column_device(s) for s in specs]
    print(f"[batch] {len(specs)} columns, {sum(s['n'] for s in specs)} values", flush=True)
    blobs = encode_batch(torch, codec, specs, cols)
    for s, c, b in zip(specs, cols, blobs):
        single = codec.encode(c, fixed_len=s["fixed_len"])
        assert torch.equal(single, b), f"batch != single for {s}"
        host = np_view(c, s["dtype"])
        expect = ref.encode(host, fixed_len=s["fixed_len"])
        assert np.array_equal(b.cpu().numpy(), expect), f"batch != oracle for {s}"


def make_batch(torch, codec, specs, cols, blobs):
    outs, sums, jobs, bounds = [], torch.zeros((len(specs), 3), dtype=torch.uint64,
                                               device="cuda"), [], []
    for i, (s, c, b) in enumerate(zip(specs, cols, blobs)):
        out = torch.empty_like(c)
        host = np_view(c, s["dtype"])
        lo, hi = W.filter_bounds(host) if s["n"] else (0, 0)
        bounds.append((lo, hi))
        outs.append(out)
        jobs.append(P.DecodeJob(b.data_ptr(), b.numel(), s["n"], out.data_ptr() if s["n"] else 0,
                                lo, hi, sums.data_ptr() + 24 * i))
    batch = P.leco_batch_create(codec.ctx, jobs)
    return batch, outs, sums, bounds


def check_outputs(torch, specs, cols, outs, sums, bounds, decoded=True, summed=True):
    sv = sums.cpu().numpy().view(np.uint64)
    for i, (s, c) in enumerate(zip(specs, cols)):
        if decoded:
            assert torch.equal(outs[i], c), f"decode mismatch in column {i}"
        if summed:
            host = np_view(c, s["dtype"]).astype(object)
            lo, hi = bounds[i]
            sel = host[(host >= lo) & (host < hi)]
            got = (int(sv[i, 1]) << 64) | int(sv[i, 0])
            assert (got, int(sv[i, 2])) == (int(sel.sum()) if len(sel) else 0, len(sel)), i


def test_batch_decode_filter_fused_and_graph(torch, codec):
    specs = small_specs(seed=8)
    cols = [W.make_column_device(s) for s in specs]
    blobs = [codec.encode(c, fixed_len=s["fixed_len"]) for s, c in zip(specs, cols)]
    batch, outs, sums, bounds = make_batch(torch, codec, specs, cols, blobs)
    try:
        for op in (P.LECO_BATCH_DECODE, P.LECO_BATCH_FILTER, P.LECO_BATCH_DECODE | P.LECO_BATCH_FILTER):
            for o in outs:
                o.zero_()
            sums.fill_(7)
            codec.check("leco_batch_run", P.leco_batch_run(batch, op))
            codec.sync()
            check_outputs(torch, specs, cols, outs, sums, bounds,
                          decoded=bool(op & 1), summed=bool(op & 2))
        # graph replays, with eager work and synchronisation between them
        for rep in range(3):
            for o in outs:
                o.fill_(rep + 1)
            sums.fill_(rep + 5)
            torch.cuda.synchronize()
            codec.check("leco_batch_run_graph", P.leco_batch_run_graph(batch, 3))
            codec.sync()
            check_outputs(torch, specs, cols, outs, sums, bounds)
    finally:
        P.leco_batch_destroy(batch)


def test_batch_decode_short_partitions(torch, codec):
    """Columns of short partitions (variable lengths 1..80, fixed L = 24):
    the batched decoder's pieces cross partition boundaries within a round."""
    rng = np.random.default_rng(17)
    specs, cols, blobs = [], [], []
    for i, (n, dtype) in enumerate([(30_000, np.uint64), (25_001, np.uint32), (9_000, np.uint64),
                                    (40_000, np.uint32)]):
        host = W.linear_noise(n, 80 + i, dtype) if i % 2 else W.constant_runs(n, 80 + i).astype(dtype)
        c = torch.from_numpy(host).cuda()
        if i < 2:
            s = [0]
            while s[-1] < n:
                s.append(min(n, s[-1] + int(rng.integers(1, 81))))
            blobs.append(codec.encode(c, starts=np.array(s, np.uint64)))
        else:
            blobs.append(codec.encode(c, fixed_len=24))
        specs.append(dict(n=n, dtype=dtype))
        cols.append(c)
    batch, outs, sums, bounds = make_batch(torch, codec, specs, cols, blobs)
    try:
        for tl in (0, 10, 14):
            codec.check("set_shape", P.leco_batch_set_shape(batch, tl, 0))
            for op in (P.LECO_BATCH_DECODE, P.LECO_BATCH_DECODE | P.LECO_BATCH_FILTER):
                for o in outs:
                    o.zero_()
                codec.check("leco_batch_run", P.leco_batch_run(batch, op))
                codec.sync()
                check_outputs(torch, specs, cols, outs, sums, bounds, summed=bool(op & 2))
    finally:
        P.leco_batch_destroy(batch)


def test_every_launch_shape_gives_identical_results(torch, codec):
    specs = small_specs(ncols=24, seed=9)
    cols = [W.make_column_device(s) for s in specs]
    blobs = [codec.encode(c, fixed_len=s["fixed_len"]) for s, c in zip(specs, cols)]
    batch, outs, sums, bounds = make_batch(torch, codec, specs, cols, blobs)
    try:
        for tl in (0, 9, 11, 12, 13, 14):
            for bpc in (0, 1, 4, 8):
                print(f"[shape] tile_log2={tl} blocks_per_cu={bpc}", flush=True)
                codec.check("set_shape", P.leco_batch_set_shape(batch, tl, bpc))
                for o in outs:
                    o.zero_()
                codec.check("leco_batch_run", P.leco_batch_run(batch, 3))
                codec.sync()
                check_outputs(torch, specs, cols, outs, sums, bounds)
        st, tl, bpc = P.leco_batch_tune(batch, 3)
        codec.check("leco_batch_tune", st)
        # one workgroup per tile, or a persistent grid of the resident count
        assert tl in (0, 12, 13, 14) and 0 <= bpc <= 64
        codec.check("leco_batch_run", P.leco_batch_run(batch, 3))
        codec.sync()
        check_outputs(torch, specs, cols, outs, sums, bounds)
    finally:
        P.leco_batch_destroy(batch)


def test_batch_rejects_mismatched_length(torch, codec):
    col = W.linear_noise_device(5000, 3, np.uint64)
    blob = codec.encode(col, fixed_len=1024)
    out = torch.empty_like(col)
    batch = P.leco_batch_create(codec.ctx, [P.DecodeJob(blob.data_ptr(), blob.numel(), 4999,
                                                        out.data_ptr(), 0, 0, 0)])
    try:
        assert P.leco_batch_run(batch, P.LECO_BATCH_DECODE) == P.LECO_OK
        assert P.leco_sync(codec.ctx) == P.LECO_EFORMAT
    finally:
        P.leco_batch_destroy(batch)


def test_tuner_cache_file(torch, codec, tmp_path):
    """The tuner's choice is kept per device, op and batch shape in a JSON
    file: the first call tunes and writes it, the second (same shape) reads
    it back without tuning, another op or shape gets its own member, and
    results are unchanged."""
    import json
    specs = small_specs(ncols=16, seed=10)
    cols = [W.make_column_device(s) for s in specs]
    blobs = [codec.encode(c, fixed_len=s["fixed_len"]) for s, c in zip(specs, cols)]
    batch, outs, sums, bounds = make_batch(torch, codec, specs, cols, blobs)
    path = str(tmp_path / "tune.json")
    try:
        st, tl, bpc, hit = P.leco_batch_tune_cached(batch, 3, path)
        codec.check("tune_cached", st)
        assert not hit
        cache = json.load(open(path))
        assert len(cache) == 1
        (key, val), = cache.items()
        assert val == {"tile_log2": tl, "blocks_per_cu": bpc} and "op3" in key
        codec.check("set_shape", P.leco_batch_set_shape(batch, 9, 1))
        st, tl2, bpc2, hit = P.leco_batch_tune_cached(batch, 3, path)
        codec.check("tune_cached", st)
        assert hit and (tl2, bpc2) == (tl, bpc)
        st, _, _, hit = P.leco_batch_tune_cached(batch, 1, path)
        assert st == P.LECO_OK and not hit and len(json.load(open(path))) == 2
        for o in outs:
            o.zero_()
        codec.check("leco_batch_run", P.leco_batch_run(batch, 3))
        codec.sync()
        check_outputs(torch, specs, cols, outs, sums, bounds)
    finally:
        P.leco_batch_destroy(batch)
    # a different batch shape is a different member
    batch2, outs2, sums2, bounds2 = make_batch(torch, codec, specs[:8], cols[:8], blobs[:8])
    try:
        st, _, _, hit = P.leco_batch_tune_cached(batch2, 3, path)
        assert st == P.LECO_OK and not hit and len(json.load(open(path))) == 3
    finally:
        P.leco_batch_destroy(batch2)
