"""Served mode on the GPU: resident compressed columns, a request loop with
admission by output memory, steps overlapped on several streams.  Every
result must equal the column's values, and be the same alone and in the
mix (tolerance 0: integers)."""
from __future__ import annotations

import time

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


@pytest.fixture(scope="module")
def columns(torch, codec):
    specs = [dict(kind="linear_noise", n=1_000_000, dtype=np.uint64, seed=3, fixed_len=1024),
             dict(kind="lognormal_keys", n=1_500_007, dtype=np.uint64, seed=4, fixed_len=4096),
             dict(kind="lognormal_keys", n=700_001, dtype=np.uint32, seed=5, fixed_len=4096),
             dict(kind="linear_noise", n=333_333, dtype=np.uint32, seed=6, fixed_len=1000)]
    cols, blobs, hosts = [], [], []
    for s in specs:
        c = W.make_column_device(s)
        cols.append(c)
        blobs.append(codec.encode(c, fixed_len=s["fixed_len"]))
        hosts.append(c.cpu().numpy().view(np.uint32 if s["dtype"] == np.uint32 else np.uint64))
    return specs, cols, blobs, hosts


def start(codec, columns, budget=256 << 20, streams=2, inflight=1024):
    specs, cols, blobs, hosts = columns
    res = [P.ResidentCol(b.data_ptr(), b.numel(), s["n"]) for s, b in zip(specs, blobs)]
    cfg = P.ServerConfig(budget, inflight, streams, 1 << 16, 1 << 20, 32 << 20, 100, 0, 16 << 20)
    return P.leco_server_start(codec.ctx, res, cfg)


def to_request(r):
    if r["kind"] == "ra":
        pos = np.ascontiguousarray(r["positions"], dtype=np.uint64)
        return P.Request(P.LECO_REQ_RANDOM_ACCESS, r["col"], pos.ctypes.data, len(pos), 0, 0), pos
    return P.Request(P.LECO_REQ_RANGE, r["col"], None, 0, r["begin"], r["end"]), None


def fetch(torch, codec, comp):
    """Copies a completion's result (device memory owned by the server,
    aligned to the value width) to the host through the library's plain
    copy kernel, from the 16-byte boundary below it."""
    nbytes = comp.count * comp.dtype
    assert comp.out_dev % comp.dtype == 0
    head = comp.out_dev % 16
    padded = (head + nbytes + 15) // 16 * 16
    buf = torch.empty(max(padded, 16), dtype=torch.uint8, device="cuda")
    if nbytes:
        lib = P.lib()
        assert lib.leco_diag_copy(codec.ctx, comp.out_dev - head, buf.data_ptr(), padded,
                                  torch.cuda.current_stream().cuda_stream) == P.LECO_OK
    torch.cuda.synchronize()
    return buf[head: head + nbytes].cpu().numpy().view(
        np.uint32 if comp.dtype == 4 else np.uint64).copy()


def expected(r, hosts):
    h = hosts[r["col"]]
    if r["kind"] == "ra":
        return h[r["positions"].astype(np.int64)]
    return h[r["begin"]: r["end"]]


def run_all(torch, codec, server, reqs, release=True, built=None):
    """Submits every request at once (as built Request structs when given)
    and collects results by ticket."""
    keep, tickets = [], {}
    for i, r in enumerate(reqs):
        if built is None:
            req, pos = to_request(r)
            keep.append(pos)
        else:
            req = built[i]
        st, t = P.leco_server_submit(server, req)
        assert st == P.LECO_OK, P.leco_last_error(codec.ctx)
        tickets[t] = i
    out = {}
    deadline = time.time() + 60
    while len(out) < len(reqs):
        assert time.time() < deadline, "server did not complete the requests"
        for c in P.leco_server_poll(server):
            assert c.status == P.LECO_OK
            out[tickets[c.ticket]] = fetch(torch, codec, c)
            if release:
                assert P.leco_server_release(server, c.ticket) == P.LECO_OK
    return out


def test_mixed_requests_equal_the_column(torch, codec, columns):
    specs, cols, blobs, hosts = columns
    reqs = W.request_mix(300, [s["n"] for s in specs], seed=61, max_log2_k=13, range_exp=(1, 5.5))
    server = start(codec, columns)
    try:
        got = run_all(torch, codec, server, reqs)
        for i, r in enumerate(reqs):
            assert np.array_equal(got[i], expected(r, hosts)), f"request {i} {r['kind']}"
        st = P.leco_server_stats_get(server)
        assert st["completed"] == len(reqs) and st["out_bytes_in_use"] == 0
    finally:
        P.leco_server_stop(server)
    assert codec.sync() is None


def device_positions(torch, reqs):
    """Random-access requests with their positions in device memory."""
    devs = [torch.from_numpy(np.ascontiguousarray(r["positions"], dtype=np.uint64).view(np.int64)).cuda()
            for r in reqs]
    torch.cuda.synchronize()
    built = [P.Request(P.LECO_REQ_RANDOM_ACCESS_DEV, r["col"], d.data_ptr(), d.numel(), 0, 0)
             for r, d in zip(reqs, devs)]
    return built, devs


def test_device_positions_match_host_positions(torch, codec, columns):
    """Positions read in place from device memory give the same results as
    positions copied from host memory, at lane-count edges (1, 255, 256, 257)
    and across several workgroups, for both widths."""
    specs, cols, blobs, hosts = columns
    rng = np.random.default_rng(64)
    reqs = [dict(kind="ra", col=c, positions=rng.integers(0, specs[c]["n"], size=k, dtype=np.uint64))
            for c in range(len(specs)) for k in (1, 255, 256, 257, 5000)]
    reqs[0]["positions"][0] = specs[0]["n"] - 1
    server = start(codec, columns)
    try:
        host = run_all(torch, codec, server, reqs)
        built, devs = device_positions(torch, reqs)
        got = run_all(torch, codec, server, reqs, built=built)
        for i, r in enumerate(reqs):
            assert np.array_equal(got[i], expected(r, hosts)), f"request {i}"
            assert np.array_equal(got[i], host[i])
        # and mixed with ranges and host-position requests in the same steps
        mix = W.request_mix(80, [s["n"] for s in specs], seed=65, max_log2_k=11, range_exp=(1, 4.5))
        mb, mdevs, keep = [], [], []
        for j, r in enumerate(mix):
            if r["kind"] == "ra" and j % 2:
                b, d = device_positions(torch, [r])
                mb.append(b[0])
                mdevs += d
            else:
                req, pos = to_request(r)
                mb.append(req)
                keep.append(pos)
        got = run_all(torch, codec, server, mix, built=mb)
        for i, r in enumerate(mix):
            assert np.array_equal(got[i], expected(r, hosts)), f"mixed request {i}"
    finally:
        P.leco_server_stop(server)
    assert codec.sync() is None


def test_device_positions_out_of_range_raise_the_flag(torch, codec, columns):
    specs, cols, blobs, hosts = columns
    n = specs[1]["n"]
    reqs = [dict(kind="ra", col=1, positions=np.array([5, n, 7], dtype=np.uint64))]
    server = start(codec, columns)
    try:
        built, devs = device_positions(torch, reqs)
        got = run_all(torch, codec, server, reqs, built=built)
        assert got[0][0] == hosts[1][5] and got[0][1] == 0 and got[0][2] == hosts[1][7]
    finally:
        P.leco_server_stop(server)
    with pytest.raises(P.LecoError) as e:
        codec.sync()
    assert e.value.status == P.LECO_ERANGE
    assert codec.sync() is None  # the flag is cleared once reported


def test_alone_equals_in_the_mix(torch, codec, columns):
    specs, cols, blobs, hosts = columns
    reqs = W.request_mix(120, [s["n"] for s in specs], seed=62, max_log2_k=12, range_exp=(1, 5))
    server = start(codec, columns, streams=3)
    try:
        mixed = run_all(torch, codec, server, reqs)
        for i in range(0, len(reqs), 3):
            alone = run_all(torch, codec, server, [reqs[i]])[0]
            assert np.array_equal(alone, mixed[i]), f"request {i} differs alone"
    finally:
        P.leco_server_stop(server)


def test_admission_respects_output_budget(torch, codec, columns):
    specs, cols, blobs, hosts = columns
    reqs = [dict(kind="range", col=1, begin=b, end=b + 60_000) for b in range(0, 1_200_000, 60_000)]
    budget = 1 << 20  # two 480 KB results fit at a time
    server = start(codec, columns, budget=budget, streams=2)
    try:
        got = run_all(torch, codec, server, reqs)
        for i, r in enumerate(reqs):
            assert np.array_equal(got[i], expected(r, hosts))
        st = P.leco_server_stats_get(server)
        assert 0 < st["out_bytes_peak"] <= budget
        assert st["steps"] >= len(reqs) // 2
    finally:
        P.leco_server_stop(server)


def test_held_results_block_admission_until_released(torch, codec, columns):
    specs, cols, blobs, hosts = columns
    server = start(codec, columns, budget=1 << 20, inflight=2)
    try:
        req = P.Request(P.LECO_REQ_RANGE, 0, None, 0, 0, 1000)
        tickets = [P.leco_server_submit(server, req)[1] for _ in range(3)]
        comps = []
        deadline = time.time() + 10
        while len(comps) < 2 and time.time() < deadline:
            comps += P.leco_server_poll(server)
        time.sleep(0.05)
        comps += P.leco_server_poll(server)
        assert len(comps) == 2, "the third request must wait for a free in-flight slot"
        assert P.leco_server_release(server, comps[0].ticket) == P.LECO_OK
        deadline = time.time() + 10
        while len(comps) < 3 and time.time() < deadline:
            comps += P.leco_server_poll(server)
        assert sorted(c.ticket for c in comps) == sorted(tickets)
    finally:
        P.leco_server_stop(server)


def test_submit_errors(torch, codec, columns):
    specs, cols, blobs, hosts = columns
    server = start(codec, columns, budget=1 << 16)
    try:
        bad = np.array([0, specs[0]["n"]], dtype=np.uint64)
        st, _ = P.leco_server_submit(server, P.Request(P.LECO_REQ_RANDOM_ACCESS, 0, bad.ctypes.data, 2, 0, 0))
        assert st == P.LECO_ERANGE
        st, _ = P.leco_server_submit(server, P.Request(P.LECO_REQ_RANGE, 9, None, 0, 0, 10))
        assert st == P.LECO_EINVAL
        st, _ = P.leco_server_submit(server, P.Request(P.LECO_REQ_RANGE, 0, None, 0, 0, 100_000))
        assert st == P.LECO_ENOSPC
        assert P.leco_server_release(server, 12345) == P.LECO_EINVAL
    finally:
        P.leco_server_stop(server)


def test_submit_batch_queues_the_accepted_prefix(torch, codec, columns):
    """One batch call queues requests in order up to the first bad one,
    whose status it returns; the accepted ones complete normally."""
    specs, cols, blobs, hosts = columns
    reqs = W.request_mix(40, [s["n"] for s in specs], seed=66, max_log2_k=10, range_exp=(1, 4))
    arr = (P.Request * (len(reqs) + 1))()
    keep = []
    for i, r in enumerate(reqs[:25]):
        arr[i], pos = to_request(r)
        keep.append(pos)
    arr[25] = P.Request(P.LECO_REQ_RANGE, 0, None, 0, 0, specs[0]["n"] + 1)  # outside [0, n)
    for i, r in enumerate(reqs[25:]):
        arr[26 + i], pos = to_request(r)
        keep.append(pos)
    server = start(codec, columns)
    try:
        st, tickets = P.leco_server_submit_batch(server, arr)
        assert st == P.LECO_ERANGE and len(tickets) == 25
        index = {t: i for i, t in enumerate(tickets)}
        got = {}
        deadline = time.time() + 30
        while len(got) < 25:
            assert time.time() < deadline
            for c in P.leco_server_poll(server):
                got[index[c.ticket]] = fetch(torch, codec, c)
                assert P.leco_server_release(server, c.ticket) == P.LECO_OK
        for i in range(25):
            assert np.array_equal(got[i], expected(reqs[i], hosts)), f"request {i}"
        st, tickets = P.leco_server_submit_batch(server, (P.Request * 0)())
        assert st == P.LECO_OK and tickets == []
    finally:
        P.leco_server_stop(server)


def test_open_loop_replay_reports_latencies(torch, codec, columns):
    specs, cols, blobs, hosts = columns
    reqs = W.request_mix(200, [s["n"] for s in specs], seed=63, max_log2_k=10, range_exp=(1, 4),
                         rate=20_000.0)
    arr = (P.Request * len(reqs))()
    keep = []
    for i, r in enumerate(reqs):
        arr[i], pos = to_request(r)
        keep.append(pos)
    arrival = np.array([r["t"] for r in reqs]) - reqs[0]["t"]
    lat = np.zeros(len(reqs))
    server = start(codec, columns)
    try:
        st, elapsed = P.leco_server_replay(server, arr, arrival, lat)
        assert st == P.LECO_OK
        assert np.all(lat > 0) and elapsed > 0
    finally:
        P.leco_server_stop(server)


def test_polynomial_blobs_are_served(torch, codec):
    """Resident columns encoded with the polynomial regressor: lookups and
    range scans equal the columns."""
    hosts_np = [W.cosmos(400_000, 71), W.poly_blocks(300_003, 72)]
    specs = [dict(n=len(h)) for h in hosts_np]
    cols = [torch.from_numpy(h).cuda() for h in hosts_np]
    blobs = [codec.encode(c, fixed_len=1000, regressor="poly") for c in cols]
    columns = (specs, cols, blobs, hosts_np)
    reqs = W.request_mix(120, [s["n"] for s in specs], seed=73, max_log2_k=12, range_exp=(1, 5.3))
    server = start(codec, columns)
    try:
        got = run_all(torch, codec, server, reqs)
        for i, r in enumerate(reqs):
            assert np.array_equal(got[i], expected(r, hosts_np)), f"request {i} {r['kind']}"
    finally:
        P.leco_server_stop(server)
    assert codec.sync() is None


def test_short_partition_blobs_are_served(torch, codec):
    """Resident columns of short partitions (variable lengths 1..100 and
    fixed L = 30): lookups and range scans equal the columns."""
    rng = np.random.default_rng(74)
    hosts_np = [W.constant_runs(300_000, 75).astype(np.uint64), W.linear_noise(200_003, 76, np.uint32)]
    specs = [dict(n=len(h)) for h in hosts_np]
    cols = [torch.from_numpy(h).cuda() for h in hosts_np]
    s = [0]
    while s[-1] < len(hosts_np[0]):
        s.append(min(len(hosts_np[0]), s[-1] + int(rng.integers(1, 101))))
    blobs = [codec.encode(cols[0], starts=np.array(s, np.uint64)), codec.encode(cols[1], fixed_len=30)]
    columns = (specs, cols, blobs, hosts_np)
    reqs = W.request_mix(120, [s["n"] for s in specs], seed=77, max_log2_k=12, range_exp=(1, 5.3))
    server = start(codec, columns)
    try:
        got = run_all(torch, codec, server, reqs)
        for i, r in enumerate(reqs):
            assert np.array_equal(got[i], expected(r, hosts_np)), f"request {i} {r['kind']}"
    finally:
        P.leco_server_stop(server)
    assert codec.sync() is None
