"""Benchmark of the LeCo hot path on one MI355X.

Workload (sorted 64-bit keys): 200,000,000 uint64 keys, the cumulative sum
of max(1, rint(lognormal(3, 1.5))) gaps (seed 2), fixed partitions of 4096
values, and 100,000,000 uniform random positions (seed 21).  The column is
encoded once on the GPU (and checked against the input); a step is one
decode_all of the whole column plus one random_access of all positions, with
inputs and blob resident in HBM.

Prints one JSON line.  `value` is decoded output GB/s of decode_all, from
HIP events around each decode_all launch on the stream it runs on;
`roofline` prices that kernel's algorithmic bytes (compressed bytes read
plus output bytes written) against the 8 TB/s HBM peak.  `cpu_baseline`
times the CPU oracle on the first 100,663,296 values of the same column.

After that step the default run frees its buffers and adds two more
workloads to the same line: `batched` (4,096 columns of lognormal lengths,
about 2e9 values, one persistent decode launch, against one decode_all
launch per column) and `served` (64 resident columns, 20 GB, a Poisson
stream of mixed lookups and range scans through the served loop, against
the same stream served one launch per request), each with its roofline
fraction, and the served one with p50/p99 latency and the host/device time
split of its request loop.  `--c2-only` skips them.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK = 8.0e12  # MI355X HBM3E, bytes/s
HOST_CPUS_PER_GPU = 16  # host CPU share of one GPU on the benchmark machines


def log(msg: str):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=200_000_000)
    ap.add_argument("--lookups", type=int, default=100_000_000)
    ap.add_argument("--cpu-sample", type=int, default=24 * 4096 * 1024)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", choices=["sorted_keys", "batched", "served", "variable",
                                           "encode_options", "higher_order", "encode_latency"],
                    default="sorted_keys")
    ap.add_argument("--var-n", type=int, default=100_000_000)
    ap.add_argument("--tau", type=float, default=0.03,
                    help="variable workload: split threshold factor (section 3.2.2)")
    ap.add_argument("--cols", type=int, default=4096)
    ap.add_argument("--served-n", type=int, default=39_062_500)
    ap.add_argument("--requests", type=int, default=20_000)
    ap.add_argument("--served-streams", type=int, default=8,
                    help="served workload: step streams")
    ap.add_argument("--served-min-step-mb", type=int, default=64,
                    help="served workload: result MiB that make a step worth launching early")
    ap.add_argument("--served-inflight", type=int, default=2048,
                    help="served workload: admitted, unreleased requests at most")
    ap.add_argument("--no-plain", action="store_true",
                    help="batched: skip the 4096-launch per-column comparison (for profiler runs)")
    ap.add_argument("--sat-requests", type=int, default=60_000,
                    help="served workload: requests of the closed-loop saturation run")
    ap.add_argument("--c2-only", action="store_true",
                    help="default run: only the sorted-keys step, without the batched and served "
                         "workloads")
    return ap.parse_args()


DECODER_SOURCES = ["paper_2306_15374_amd/csrc/decode.hip", "paper_2306_15374_amd/csrc/decode_tile.hpp",
                   "paper_2306_15374_amd/csrc/leco_dev.hpp"]
TRAFFIC_PROFILE = "profiles/k_decode_sorted_keys_200M.md"
BATCH_SOURCES = ["paper_2306_15374_amd/csrc/batch.hip", "paper_2306_15374_amd/csrc/decode_tile.hpp",
                 "paper_2306_15374_amd/csrc/leco_dev.hpp"]
BATCH_TRAFFIC_PROFILE = "profiles/k_batch_decode_4096_columns.md"


def measured_traffic(sources=DECODER_SOURCES, profile=TRAFFIC_PROFILE):
    """HBM bytes per launch from a committed rocprofv3 counter summary, or
    None if the kernel's sources changed since it was taken."""
    import hashlib
    try:
        h = hashlib.sha256()
        for f in sources:
            h.update(open(os.path.join(ROOT, f), "rb").read())
        for line in open(os.path.join(ROOT, profile)):
            line = line.strip()
            if line.startswith("{") and '"source_sha"' in line:
                rec = json.loads(line)
                if rec["source_sha"] == h.hexdigest()[:16]:
                    return rec["traffic_bytes"]
    except OSError:
        pass
    return None


def cpu_baseline(col: np.ndarray, pos: np.ndarray, sample: int, L: int, gpu_blob: np.ndarray):
    """Times the oracle (single thread) on the first `sample` values and
    checks the GPU blob's leading partitions against the oracle's bytes."""
    import oracle
    sample = min(sample, len(col)) // L * L
    part = col[:sample]
    t0 = time.perf_counter()
    blob = oracle.encode(part, fixed_len=L)
    t_enc = time.perf_counter() - t0
    t0 = time.perf_counter()
    dec = oracle.decode_all(blob)
    t_dec = time.perf_counter() - t0
    assert np.array_equal(dec, part)
    p = pos[pos < sample][:2_000_000]
    t0 = time.perf_counter()
    ra = oracle.random_access(blob, p)
    t_ra = time.perf_counter() - t0
    assert np.array_equal(ra, part[p])
    # prefix parity: records and words of the sampled partitions
    m = sample // L
    hdr = blob[:64].view(np.uint64)
    words_off, tw = int(hdr[6]), int(hdr[7])
    ghdr = gpu_blob[:64].view(np.uint64)
    g_words_off = int(ghdr[6])
    assert np.array_equal(gpu_blob[64: 64 + 32 * m], blob[64: 64 + 32 * m]), "record parity"
    assert np.array_equal(gpu_blob[g_words_off: g_words_off + 8 * tw],
                          blob[words_off: words_off + 8 * tw]), "word parity"
    # the same sample on every host core: static chunks of whole partitions,
    # one oracle call per chunk and thread (the C calls release the GIL)
    from concurrent.futures import ThreadPoolExecutor
    host = host_facts()
    # one thread per CPU the process may use, within its cgroup quota and the
    # host share of one GPU on this machine (16 CPUs per GPU)
    cap = min(host["usable_cpus"], int(host["cgroup_cpus"] or host["usable_cpus"]), HOST_CPUS_PER_GPU)
    cores = max(1, min(cap, m))
    bounds = [(m * i // cores) * L for i in range(cores + 1)]
    chunks = [part[bounds[i]:bounds[i + 1]] for i in range(cores)]
    with ThreadPoolExecutor(cores) as ex:
        t0 = time.perf_counter()
        blobs = list(ex.map(lambda c: oracle.encode(c, fixed_len=L), chunks))
        t_enc_mt = time.perf_counter() - t0
        t0 = time.perf_counter()
        outs = list(ex.map(oracle.decode_all, blobs))
        t_dec_mt = time.perf_counter() - t0
    assert all(np.array_equal(o, c) for o, c in zip(outs, chunks))
    return dict(value=sample * 8 / t_dec_mt / 1e9, unit="GB/s", cores=cores, kind="oracle",
                nproc=host["nproc"], usable_cpus=host["usable_cpus"],
                cgroup_cpus=host["cgroup_cpus"], cpu_model=host["cpu_model"],
                sample=f"first {sample} values ({m} partitions of {L}) in {cores} static chunks, "
                       f"one thread each: decode_all {t_dec_mt:.2f} s, encode {t_enc_mt:.2f} s; "
                       f"one thread: decode_all {t_dec:.2f} s; encode {t_enc:.2f} s; "
                       f"random_access of {len(p)} positions {t_ra:.2f} s "
                       f"({len(p) / t_ra:.3e} lookups/s)",
                encode_GBps=sample * 8 / t_enc_mt / 1e9, lookups_per_s=len(p) / t_ra,
                single_thread={"decode_GBps": sample * 8 / t_dec / 1e9,
                               "encode_GBps": sample * 8 / t_enc / 1e9,
                               "lookups_per_s": len(p) / t_ra})


def host_facts() -> dict:
    """Host CPU facts for the CPU baseline: nproc, the CPUs this process may
    run on, and the model string from /proc/cpuinfo."""
    nproc = os.cpu_count() or 1
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = nproc
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    quota = None  # CPUs granted by the cgroup's cpu.max, if it sets one
    try:
        q, period = open("/sys/fs/cgroup/cpu.max").read().split()[:2]
        if q != "max":
            quota = int(q) / int(period)
    except (OSError, ValueError):
        pass
    return {"nproc": nproc, "usable_cpus": usable, "cgroup_cpus": quota, "cpu_model": model}


def time_events(torch, stream, fn, reps: int) -> float:
    """Median seconds of fn() over reps runs, HIP events on `stream`."""
    ts = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        fn()
        b.record(stream)
        torch.cuda.synchronize()
        ts.append(a.elapsed_time(b) / 1e3)
    return float(np.median(ts))


def time_stream(torch, stream, fn, reps: int) -> float:
    """Mean seconds of fn() over reps launches back to back on `stream`,
    between two HIP events (the launches queue while earlier ones run, as
    in a loop of calls; the kernel profiler's durations compare to this)."""
    fn()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(reps):
        fn()
    b.record(stream)
    torch.cuda.synchronize()
    return a.elapsed_time(b) / 1e3 / reps


def bench_batched(args, codec=None):
    """4,096 columns (lognormal lengths 1e3..1e7, ~2.0e9 values, half uint32)
    encoded in one launch sequence and decoded in one persistent launch,
    against the plain path of one decode_all launch per column on one
    stream.  Returns the result dict."""
    import torch
    import paper_2306_15374_amd as P
    from paper_2306_15374_amd import workloads as W

    specs = W.batched_columns(args.cols)
    own = codec is None
    codec = codec or P.Codec(0)
    stream = torch.cuda.current_stream()
    log(f"batched: drawing {len(specs)} columns on the device")
    cols = [W.make_column_device(s) for s in specs]
    n_total = sum(s["n"] for s in specs)
    in_bytes = sum(s["n"] * (4 if s["dtype"] == np.uint32 else 8) for s in specs)
    bufs, jobs = [], []
    sizes = torch.zeros(len(specs), dtype=torch.uint64, device="cuda")
    for i, (s, c) in enumerate(zip(specs, cols)):
        dt = P.LECO_U32 if s["dtype"] == np.uint32 else P.LECO_U64
        part, _ = P.make_partitioning(fixed_len=s["fixed_len"])
        cap = P.leco_max_blob_bytes(s["n"], dt, part)
        buf = torch.empty(cap, dtype=torch.uint8, device="cuda")
        bufs.append(buf)
        jobs.append(P.EncodeJob(c.data_ptr(), s["n"], dt, 0, s["fixed_len"], buf.data_ptr(), cap,
                                sizes.data_ptr() + 8 * i))
    torch.cuda.synchronize()
    log(f"batched: {n_total} values, {in_bytes / 1e9:.2f} GB; batched encode")
    enc = lambda: codec.check("leco_encode_batch", P.leco_encode_batch(codec.ctx, jobs))
    enc()
    codec.sync()
    t_enc = time_events(torch, stream, enc, 5)
    codec.sync()
    sz = sizes.cpu().numpy().view(np.uint64)
    blob_total = int(sz.sum())
    blobs = [b[: int(n)] for b, n in zip(bufs, sz)]
    # every column round-trips; sampled columns match single-column encodes
    outs = [torch.empty_like(c) for c in cols]
    sums = torch.zeros((len(specs), 3), dtype=torch.uint64, device="cuda")
    djobs = []
    for i, (s, c, b) in enumerate(zip(specs, cols, blobs)):
        djobs.append(P.DecodeJob(b.data_ptr(), b.numel(), s["n"], outs[i].data_ptr(), 0, 0,
                                 sums.data_ptr() + 24 * i))
    # filter bounds [vmin + R/4, vmin + 3R/4) per column (computed on the device)
    for i, c in enumerate(cols):
        vmin, vmax = int(c.min()), int(c.max())
        r = vmax - vmin
        djobs[i].lo, djobs[i].hi = vmin + r // 4, vmin + (3 * r) // 4
    batch = P.leco_batch_create(codec.ctx, djobs)
    st, tl, bpc = P.leco_batch_tune(batch, P.LECO_BATCH_DECODE)
    codec.check("leco_batch_tune", st)
    log(f"batched: tuned shape: tile {'per column' if tl == 0 else f'2^{tl}'}, blocks/CU {bpc}")
    run = lambda op: (lambda: codec.check("leco_batch_run", P.leco_batch_run(batch, op)))
    run(P.LECO_BATCH_DECODE)()
    codec.sync()
    for s, c, o in zip(specs, cols, outs):
        assert torch.equal(o, c), f"batched decode mismatch {s}"
    for i in range(0, len(specs), 97):
        assert torch.equal(blobs[i], codec.encode(cols[i], fixed_len=specs[i]["fixed_len"]))
    t_dec = time_events(torch, stream, run(P.LECO_BATCH_DECODE), args.steps)
    t_graph = time_events(torch, stream, lambda: codec.check(
        "graph", P.leco_batch_run_graph(batch, P.LECO_BATCH_DECODE)), args.steps)
    t_filter = time_events(torch, stream, run(P.LECO_BATCH_FILTER), args.steps)
    t_fused = time_events(torch, stream, run(P.LECO_BATCH_DECODE | P.LECO_BATCH_FILTER), args.steps)
    codec.sync()
    # filter sums against torch on the decoded columns
    sv = sums.cpu().numpy().view(np.uint64)
    for i in range(0, len(specs), 61):
        c = cols[i]
        sel = c[(c >= djobs[i].lo) & (c < djobs[i].hi)]
        assert int(sv[i, 2]) == sel.numel() and \
            ((int(sv[i, 1]) << 64) | int(sv[i, 0])) == int(sel.to(torch.int64).sum())

    def plain():
        for b, o, s in zip(blobs, outs, specs):
            codec.check("leco_decode_all", P.leco_decode_all(codec.ctx, b, b.numel(), o, s["n"]))
    t_plain = None
    if not args.no_plain:
        plain()
        codec.sync()
        for s, c, o in zip(specs, cols, outs):
            assert torch.equal(o, c), f"plain decode mismatch {s}"
        t_plain = time_events(torch, stream, plain, 3)
    codec.sync()
    P.leco_batch_destroy(batch)
    alg = blob_total + in_bytes
    res = {
        "metric": "decoded GB/s + lookups/s vs HBM roofline (batched/served vs plain); p99 latency",
        "value": round(in_bytes / t_dec / 1e9, 2), "unit": "GB/s decoded (batched decode)",
        "n_gpus": 1, "steps": args.steps, "warmup": 1, "ms_per_step": round(t_dec * 1e3, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32+u64",
        "data": "synthetic (device-drawn linear-noise and lognormal-key columns)",
        "config": {"workload": f"batched: {len(specs)} columns, {n_total} values "
                               f"({in_bytes / 1e9:.2f} GB), lognormal lengths 1e3..1e7",
                   "tile_log2": tl, "blocks_per_cu": bpc},
        "batched_decode_ms": round(t_dec * 1e3, 3),
        "batched_decode_graph_ms": round(t_graph * 1e3, 3),
        "plain_per_column_decode_ms": None if t_plain is None else round(t_plain * 1e3, 3),
        "speedup_vs_plain": None if t_plain is None else round(t_plain / t_dec, 2),
        "plain_hbm_frac": None if t_plain is None else round(alg / t_plain / HBM_PEAK, 4),
        "filter_sum_ms": round(t_filter * 1e3, 3),
        "filter_sum_values_per_s": round(n_total / t_filter, 1),
        "fused_decode_filter_ms": round(t_fused * 1e3, 3),
        "batched_encode_ms": round(t_enc * 1e3, 3),
        "batched_encode_GBps": round(in_bytes / t_enc / 1e9, 2),
        "batched_encode_hbm_frac": round((in_bytes + blob_total) / t_enc / HBM_PEAK, 4),
        "compression_ratio": round(blob_total / in_bytes, 5),
        "roofline": {"bound": "hbm", "achieved": round(alg / t_dec / 1e9, 1), "peak": HBM_PEAK / 1e9,
                     "unit": "GB/s", "frac": round(alg / t_dec / HBM_PEAK, 4),
                     "traffic": (measured_traffic(BATCH_SOURCES, BATCH_TRAFFIC_PROFILE)
                                 if args.cols == 4096 else None),
                     "kernel": "k_batch_decode", "bytes_per_launch": alg},
        "cpu_baseline": None,
    }
    del cols, outs, bufs, blobs, sums, sizes
    if own:
        codec.close()
    torch.cuda.empty_cache()
    return res


def served_requests(torch, P, W, lens, num, seed, rate, device_positions=True):
    """The served request stream; random-access positions either resident
    in device memory before the run (read in place by the step kernel) or in
    host memory (copied into the server's pinned ring at submit)."""
    reqs = W.request_mix(num, lens, seed, rate=rate)
    arr = (P.Request * num)()
    keep = []
    ra = [r for r in reqs if r["kind"] == "ra"]
    if device_positions and ra:
        flat = torch.from_numpy(np.concatenate([r["positions"] for r in ra]).view(np.int64)).cuda()
        torch.cuda.synchronize()
        keep.append(flat)
        base, off = flat.data_ptr(), 0
    for i, r in enumerate(reqs):
        if r["kind"] == "ra":
            k = len(r["positions"])
            if device_positions:
                arr[i] = P.Request(P.LECO_REQ_RANDOM_ACCESS_DEV, r["col"], base + 8 * off, k, 0, 0)
                off += k
            else:
                pos = np.ascontiguousarray(r["positions"])
                keep.append(pos)
                arr[i] = P.Request(P.LECO_REQ_RANDOM_ACCESS, r["col"], pos.ctypes.data, k, 0, 0)
        else:
            arr[i] = P.Request(P.LECO_REQ_RANGE, r["col"], None, 0, r["begin"], r["end"])
    arrival = np.array([r["t"] for r in reqs]) - reqs[0]["t"]
    return reqs, arr, keep, arrival


def bench_served(args, codec=None):
    """64 resident uint64 columns of 39,062,500 values (20 GB uncompressed),
    a Poisson stream mixing random-access batches of floor(2^U[0,16])
    positions and range scans of floor(10^U[3,7]) values.  Saturation is
    measured closed-loop (all requests queued at once), then open-loop at
    0.3, 0.6 and 0.9 of it, each with p50/p99 latency; the plain path (one
    launch per request, same streams of requests) is measured the same way.
    Returns the result dict."""
    import torch
    import paper_2306_15374_amd as P
    from paper_2306_15374_amd import workloads as W

    specs = W.served_columns(args.cols if args.cols != 4096 else W.C5_COLS, args.served_n)
    own = codec is None
    codec = codec or P.Codec(0)
    log(f"served: drawing and encoding {len(specs)} columns of {specs[0]['n']} values")
    cols, blobs = [], []
    for s in specs:
        c = W.make_column_device(s)
        blobs.append(codec.encode(c, fixed_len=s["fixed_len"]))
        cols.append(c)
    compressed = sum(b.numel() for b in blobs)
    raw = sum(s["n"] * 8 for s in specs)
    ratio = compressed / raw
    res = [P.ResidentCol(b.data_ptr(), b.numel(), s["n"]) for s, b in zip(specs, blobs)]
    cfg = P.ServerConfig(8 << 30, args.served_inflight, args.served_streams, 1 << 16, 1 << 20,
                         args.served_min_step_mb << 20, 100, 0, 256 << 20)
    server = P.leco_server_start(codec.ctx, res, cfg)
    lens = [s["n"] for s in specs]
    mk = lambda num, seed, rate, dev=True: served_requests(torch, P, W, lens, num, seed, rate, dev)

    # correctness on a sample: alone results equal the resident column
    sreqs, sarr, skeep, _ = mk(64, W.C5_SEED + 7, 1.0, dev=False)
    for i, r in enumerate(sreqs):
        st, t = P.leco_server_submit(server, sarr[i])
        codec.check("submit", st)
        while True:
            comp = P.leco_server_poll(server, 1)
            if comp:
                break
        c = comp[0]
        nbytes = c.count * 8
        head = c.out_dev % 16  # results are aligned to the value width
        padded = (head + nbytes + 15) // 16 * 16
        buf = torch.empty(max(padded, 16), dtype=torch.uint8, device="cuda")
        if nbytes:
            codec.check("copy", P.leco_diag_copy(codec.ctx, c.out_dev - head, buf, padded))
        got = buf[head: head + nbytes].view(torch.int64)
        col = cols[r["col"]]
        exp = col[torch.from_numpy(r["positions"].astype(np.int64)).cuda()] if r["kind"] == "ra" \
            else col[r["begin"]: r["end"]]
        assert torch.equal(got, exp), f"served request {i} mismatch"
        P.leco_server_release(server, c.ticket)
    log("served: sampled results equal the resident columns")

    def traffic(reqs):
        lookups = sum(len(r["positions"]) for r in reqs if r["kind"] == "ra")
        scanned = sum(r["end"] - r["begin"] for r in reqs if r["kind"] == "range")
        # bytes a request moves: its values out, plus the compressed bytes
        # read (range: ratio * 8 per value; random access: one 8-byte word
        # and the 8-byte position)
        return lookups, scanned, scanned * 8 * (1 + ratio) + lookups * (8 + 8 + 8)

    def split(stats, elapsed):
        """Where the request loop's time went (per step, microseconds) and
        how much of the run the device was busy."""
        steps = max(stats["steps"], 1)
        return {"steps": stats["steps"], "items_per_step": round(stats["items"] / steps, 1),
                "requests_per_step": round(stats["completed"] / steps, 2),
                "host_us_per_step": {k: round(stats[f"host_{k}_ns"] / steps / 1e3, 2)
                                     for k in ("submit", "admit", "build", "launch", "retire", "wait")},
                "gpu_step_us_mean": round(stats["gpu_step_ns"] / steps / 1e3, 2),
                "gpu_busy_frac_of_elapsed": round(stats["gpu_busy_ns"] / 1e9 / elapsed, 4),
                "gpu_steps_in_flight_mean": round(stats["gpu_step_ns"] / max(stats["gpu_busy_ns"], 1), 2)}

    # saturation with positions in host memory (copied at submit), for reference
    num = args.requests
    hreqs, harr, hkeep, _ = mk(num, W.C5_SEED + 1, 1.0, dev=False)
    st, h_elapsed = P.leco_server_replay(server, harr, np.zeros(num), None)
    codec.check("replay", st)
    log(f"served: closed loop, host positions: {num / h_elapsed:.0f} req/s")
    del hkeep, harr, hreqs
    # the measured runs: every input (columns and positions) resident in HBM
    nsat = args.sat_requests
    reqs, arr, keep, _ = mk(nsat, W.C5_SEED + 1, 1.0)
    lookups, scanned, alg = traffic(reqs)
    lat = np.zeros(nsat)
    P.leco_server_stats_reset(server)
    st, elapsed = P.leco_server_replay(server, arr, np.zeros(nsat), lat)
    codec.check("replay", st)
    sat_split = split(P.leco_server_stats_get(server), elapsed)
    sat = nsat / elapsed
    log(f"served: closed loop: {nsat} requests in {elapsed:.3f} s = {sat:.0f} req/s, "
        f"{alg / elapsed / HBM_PEAK:.3f} of peak; {sat_split}")
    # the plain path over the same closed-loop stream
    # room for the largest request the stream can hold: 2^16 positions or a
    # range of 10^7 values
    out_bytes = 8 * max(1 << 16, 10_000_000)
    pbuf = torch.empty(out_bytes, dtype=torch.uint8, device="cuda")
    plat = np.zeros(nsat)
    st, p_elapsed = P.leco_plain_replay(codec.ctx, res, arr, np.zeros(nsat), pbuf, pbuf.numel(),
                                        latencies_out=plat)
    codec.check("plain replay", st)
    codec.sync()
    p_sat = nsat / p_elapsed
    log(f"served: plain closed loop: {p_sat:.0f} req/s, {alg / p_elapsed / HBM_PEAK:.3f} of peak")
    del keep, arr
    points, plain_points = {}, {}
    for frac in (0.3, 0.6, 0.9):
        rate = frac * sat
        reqs_f, arr_f, keep_f, arr_t = mk(args.requests, W.C5_SEED + 2 + int(frac * 10), rate)
        n_f = len(reqs_f)
        lat_f = np.zeros(n_f)
        P.leco_server_stats_reset(server)
        st, el = P.leco_server_replay(server, arr_f, arr_t, lat_f)
        codec.check("replay", st)
        _, _, alg_f = traffic(reqs_f)
        points[str(frac)] = {"offered_req_per_s": round(rate, 1), "achieved_req_per_s": round(n_f / el, 1),
                             "p50_us": round(float(np.percentile(lat_f, 50)), 1),
                             "p99_us": round(float(np.percentile(lat_f, 99)), 1),
                             "hbm_frac": round(alg_f / el / HBM_PEAK, 4),
                             "split": split(P.leco_server_stats_get(server), el)}
        log(f"served: open loop {frac}: {points[str(frac)]}")
        lat_p = np.zeros(n_f)
        st, el_p = P.leco_plain_replay(codec.ctx, res, arr_f, arr_t, pbuf, pbuf.numel(),
                                       latencies_out=lat_p)
        codec.check("plain replay", st)
        codec.sync()
        plain_points[str(frac)] = {"offered_req_per_s": round(rate, 1),
                                   "achieved_req_per_s": round(n_f / el_p, 1),
                                   "p50_us": round(float(np.percentile(lat_p, 50)), 1),
                                   "p99_us": round(float(np.percentile(lat_p, 99)), 1)}
        log(f"served: plain open loop {frac}: {plain_points[str(frac)]}")
        del keep_f, arr_f
    stats = P.leco_server_stats_get(server)
    P.leco_server_stop(server)
    codec.sync()
    out = {
        "metric": "decoded GB/s + lookups/s vs HBM roofline (batched/served vs plain); p99 latency",
        "value": round(scanned * 8 / elapsed / 1e9, 2), "unit": "GB/s decoded (served range scans, saturated)",
        "n_gpus": 1, "steps": 1, "warmup": 1, "ms_per_step": round(elapsed * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64",
        "data": "synthetic (device-drawn linear-noise and lognormal-key columns)",
        "config": {"workload": f"served: {len(specs)} resident uint64 columns x {specs[0]['n']} "
                               f"values ({raw / 1e9:.1f} GB), {nsat} mixed requests closed loop, "
                               f"{args.requests} per open-loop point",
                   "out_budget_bytes": 8 << 30, "streams": args.served_streams,
                   "max_inflight": args.served_inflight,
                   "min_step_bytes": args.served_min_step_mb << 20, "max_wait_us": 100},
        "saturation_req_per_s": round(sat, 1),
        "saturation_req_per_s_host_positions": round(num / h_elapsed, 1),
        "lookups_per_s": round(lookups / elapsed, 1),
        "scan_GBps_decoded": round(scanned * 8 / elapsed / 1e9, 2),
        "closed_loop_p50_us": round(float(np.percentile(lat, 50)), 1),
        "closed_loop_p99_us": round(float(np.percentile(lat, 99)), 1),
        "closed_loop_split": sat_split,
        "open_loop": points,
        "plain": {"saturation_req_per_s": round(p_sat, 1),
                  "hbm_frac": round(alg / p_elapsed / HBM_PEAK, 4),
                  "closed_loop_p50_us": round(float(np.percentile(plat, 50)), 1),
                  "closed_loop_p99_us": round(float(np.percentile(plat, 99)), 1),
                  "open_loop": plain_points},
        "speedup_vs_plain": round(sat / p_sat, 2),
        "steps_launched": stats["steps"],
        "compression_ratio": round(ratio, 5),
        "roofline": {"bound": "hbm", "achieved": round(alg / elapsed / 1e9, 1), "peak": HBM_PEAK / 1e9,
                     "unit": "GB/s", "frac": round(alg / elapsed / HBM_PEAK, 4), "traffic": None,
                     "kernel": "k_serve_step", "bytes_per_launch": None},
        "cpu_baseline": None,
    }
    del cols, blobs, pbuf
    if own:
        codec.close()
    torch.cuda.empty_cache()
    return out


def bench_variable(args):
    """Variable-length partitions: three uint32 columns of 1e8 values
    (sorted normal samples, a 1000-piece noisy polyline, runs of repeated
    values) partitioned on the GPU (greedy split and merge rounds), encoded
    with those partitions and decoded; sizes against fixed partitions of
    1024 and 4096 values."""
    import torch
    import paper_2306_15374_amd as P
    from paper_2306_15374_amd import workloads as W

    codec = P.Codec(0)
    stream = torch.cuda.current_stream()
    n = args.var_n
    gens = [("sorted_normal", W.sorted_normal), ("piecewise_linear", W.piecewise_linear),
            ("constant_runs", W.constant_runs)]
    per, host_cols = {}, []
    t_dec_all = alg_all = out_all = 0.0
    for (name, gen), seed in zip(gens, W.C3_SEEDS):
        log(f"{name}: drawing {n} values")
        col = gen(n, seed)
        host_cols.append(col)
        d = torch.from_numpy(col).cuda()
        torch.cuda.synchronize()
        starts, t_part = None, []
        for _ in range(3):
            t0 = time.perf_counter()
            starts = codec.partition(d, tau=args.tau)
            t_part.append(time.perf_counter() - t0)
            log(f"{name}: partitioned in {t_part[-1] * 1e3:.1f} ms, {len(starts) - 1} partitions")
        t_part = float(np.median(t_part))
        m = len(starts) - 1
        part, keep = P.make_partitioning(starts=starts)
        cap = P.leco_max_blob_bytes(n, P.LECO_U32, part)
        buf = torch.empty(cap, dtype=torch.uint8, device="cuda")
        size = torch.zeros(1, dtype=torch.uint64, device="cuda")
        enc = lambda: codec.check("leco_encode_async", P.leco_encode_async(
            codec.ctx, d, n, P.LECO_U32, part, buf, cap, size))
        enc()
        codec.sync()
        t_enc = time_stream(torch, stream, enc, args.steps)
        codec.sync()
        nbytes = int(size.cpu().numpy().view(np.uint64)[0])
        blob = buf[:nbytes]
        out = torch.empty_like(d)
        dec = lambda: codec.check("leco_decode_all", P.leco_decode_all(
            codec.ctx, blob, nbytes, out, n))
        dec()
        codec.sync()
        assert torch.equal(out, d), f"{name}: variable-partition round trip"
        t_dec = time_stream(torch, stream, dec, args.steps)
        t_dec_iso = time_events(torch, stream, dec, args.steps)
        codec.sync()
        fixed = {L: codec.encode(d, fixed_len=L).numel() for L in (1024, 4096)}
        # the split also beginning partitions at the starting positions
        t_sp = []
        for _ in range(3):
            t0 = time.perf_counter()
            starts_sp = codec.partition(d, tau=args.tau, start_positions=True)
            t_sp.append(time.perf_counter() - t0)
            log(f"{name}: with starting partitions in {t_sp[-1] * 1e3:.1f} ms")
        blob_sp = codec.encode(d, starts=starts_sp)
        lens = np.diff(starts.astype(np.int64))
        per[name] = {"partitions": m, "mean_len": round(float(lens.mean()), 1),
                     "max_len": int(lens.max()), "blob_bytes": nbytes,
                     "ratio": round(nbytes / (4 * n), 5),
                     "ratio_fixed_1024": round(fixed[1024] / (4 * n), 5),
                     "ratio_fixed_4096": round(fixed[4096] / (4 * n), 5),
                     "partition_ms": round(t_part * 1e3, 2),
                     "partition_values_per_s": round(n / t_part, 1),
                     "encode_ms": round(t_enc * 1e3, 3), "decode_all_ms": round(t_dec * 1e3, 4),
                     "decode_all_ms_isolated": round(t_dec_iso * 1e3, 4),
                     "decode_hbm_frac": round((nbytes + 4 * n) / t_dec / HBM_PEAK, 4),
                     "start_positions": {"partitions": len(starts_sp) - 1,
                                         "ratio": round(blob_sp.numel() / (4 * n), 5),
                                         "partition_ms": round(float(np.median(t_sp)) * 1e3, 2)}}
        del blob_sp
        log(f"{name}: {per[name]}")
        t_dec_all += t_dec
        alg_all += nbytes + 4 * n
        out_all += 4 * n
        del d, buf, out, blob
        torch.cuda.empty_cache()
    cpu = None
    if not args.no_cpu_baseline:
        # the oracle on the first 2^16 values of each column: its merge scan
        # refits every grown partition at each step, so a sample of 2^20
        # values of the polyline takes minutes
        import oracle
        k = min(n, 1 << 16)
        t_p = t_d = 0.0
        for col in host_cols:
            c = col[:k]
            t0 = time.perf_counter()
            st = oracle.partition_greedy(c, tau=args.tau)
            t_p += time.perf_counter() - t0
            log(f"oracle partitioned {k} values in {time.perf_counter() - t0:.2f} s")
            blob = oracle.encode(c, starts=st)
            t0 = time.perf_counter()
            assert np.array_equal(oracle.decode_all(blob), c)
            t_d += time.perf_counter() - t0
        cpu = {"value": round(3 * k * 4 / t_d / 1e9, 4), "unit": "GB/s", "cores": 1, "kind": "oracle",
               "sample": f"first {k} values of each column: greedy partitioning {t_p:.2f} s "
                         f"({3 * k / t_p:.3e} values/s), decode_all {t_d:.2f} s"}
    res = {
        "metric": "decoded GB/s + lookups/s vs HBM roofline (batched/served vs plain); p99 latency",
        "value": round(out_all / t_dec_all / 1e9, 2), "unit": "GB/s decoded (decode_all, variable partitions)",
        "n_gpus": 1, "steps": args.steps, "warmup": 1, "ms_per_step": round(t_dec_all * 1e3, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32",
        "data": "synthetic (seeded sorted-normal, noisy polyline and constant-run columns)",
        "config": {"workload": f"variable partitions: 3 uint32 columns x {n} values, "
                               f"greedy split (tau {args.tau}, S_M 320 bits) + merge rounds on the GPU"},
        "columns": per,
        "roofline": {"bound": "hbm", "achieved": round(alg_all / t_dec_all / 1e9, 1),
                     "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                     "frac": round(alg_all / t_dec_all / HBM_PEAK, 4), "traffic": None,
                     "kernel": "k_decode", "bytes_per_launch": None},
        "cpu_baseline": cpu,
    }
    print(json.dumps(res), flush=True)
    codec.close()


def bench_encode_options(args):
    """The encoder's options on two 2e8-value uint64 columns (sorted keys,
    linear noise): the fixed partition size search of section 3.2.1 on a 1%
    sample of 10,000-value windows, and the minimax regressor, each with the
    blob sizes it leads to."""
    import torch
    import paper_2306_15374_amd as P
    from paper_2306_15374_amd import workloads as W

    codec = P.Codec(0)
    stream = torch.cuda.current_stream()
    n = args.n
    cols = {}
    for name, gen, L0 in (("sorted_keys", W.lognormal_keys_device, W.C2_L),
                          ("linear_noise", W.linear_noise_device, W.C1_L)):
        log(f"{name}: generating {n} values")
        d = gen(n, 5, np.uint64)
        torch.cuda.synchronize()
        window = 10_000
        starts = W.sample_window_starts(n, window, fraction=0.01, seed=61)
        t = []
        res = None
        for _ in range(3):
            t0 = time.perf_counter()
            res = codec.size_search(d, starts, window)
            t.append(time.perf_counter() - t0)
        t_search = float(np.median(t))
        Ls = res["L"]
        sizes = {L: codec.encode(d, fixed_len=L).numel() for L in sorted({Ls, 1024, 4096})}
        part_ls, _ = P.make_partitioning(fixed_len=L0)
        part_mm, _ = P.make_partitioning(fixed_len=L0, regressor="minimax")
        cap = P.leco_max_blob_bytes(n, P.LECO_U64, part_ls)
        buf = torch.empty(cap, dtype=torch.uint8, device="cuda")
        size = torch.zeros(1, dtype=torch.uint64, device="cuda")
        enc = {}
        for reg, part in (("ls", part_ls), ("minimax", part_mm)):
            f = lambda: codec.check("leco_encode_async", P.leco_encode_async(
                codec.ctx, d, n, P.LECO_U64, part, buf, cap, size))
            f()
            codec.sync()
            ms = time_events(torch, stream, f, max(1, min(args.steps, 5))) * 1e3
            codec.sync()
            enc[reg] = {"encode_ms": round(ms, 3), "blob_bytes": int(size.item())}
        blob = codec.encode(d, fixed_len=L0, regressor="minimax")
        assert torch.equal(codec.decode_all(blob, out=torch.empty_like(d)), d), \
            f"{name}: minimax round trip"
        cols[name] = {
            "size_search": {"window": window, "windows": len(starts), "sampled_values": len(starts) * window,
                            "evaluations": len(res["trace"]), "ms": round(t_search * 1e3, 2),
                            "L": Ls, "sampled_cost": res["cost"],
                            "ratio_at_L": round(sizes[Ls] / (8 * n), 5),
                            "ratio_fixed_1024": round(sizes[1024] / (8 * n), 5),
                            "ratio_fixed_4096": round(sizes[4096] / (8 * n), 5)},
            "minimax": {"L": L0, **{f"{k}_{r}": v for r, e in enc.items() for k, v in e.items()},
                        "smaller_by_pct": round(100 * (enc["ls"]["blob_bytes"] - enc["minimax"]["blob_bytes"])
                                                / enc["ls"]["blob_bytes"], 3)},
        }
        log(f"{name}: {cols[name]}")
        del d, buf, blob
        torch.cuda.empty_cache()
    t_all = sum(c["minimax"]["encode_ms_minimax"] for c in cols.values()) / 1e3
    res = {
        "metric": "decoded GB/s + lookups/s vs HBM roofline (batched/served vs plain); p99 latency",
        "value": round(2 * 8 * n / t_all / 1e9, 2), "unit": "GB/s encoded (minimax regressor, input bytes)",
        "n_gpus": 1, "steps": args.steps, "warmup": 1, "ms_per_step": round(t_all * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64",
        "data": "synthetic (seeded lognormal-gap sorted keys, linear column with uniform noise)",
        "config": {"workload": f"encoder options: 2 uint64 columns x {n} values; size search over 1% "
                               "of the column in 10,000-value windows; minimax regressor"},
        "columns": cols,
        "roofline": None,
        "cpu_baseline": None,
    }
    print(json.dumps(res), flush=True)
    codec.close()


def bench_encode_latency(args):
    """Encode time of one sorted-key uint64 column from 1e4 to 1e8 values at
    partitions of 1024 and 4096, launches back to back on one stream: the
    default context (a one-pass encoder for launches of at most two
    workgroups per CU, else two passes) against one with the one-pass
    encoders off.  Both contexts' blobs are compared byte for byte."""
    import torch
    import paper_2306_15374_amd as P
    from paper_2306_15374_amd import workloads as W

    keys = ("LECO_ENCODE_FUSED", "LECO_ENCODE_FUSED_WAVE")
    old = {k: os.environ.get(k) for k in keys}
    auto = P.Codec(0)
    os.environ.update({k: "0" for k in keys})
    try:
        two = P.Codec(0)  # the overrides are read when a context is created
    finally:
        for k, v in old.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    stream = torch.cuda.current_stream()
    rows = []
    for L in (1024, 4096):
        for n in (10**4, 10**5, 10**6, 2 * 10**6, 3 * 10**6, 10**7, 10**8):
            d = W.lognormal_keys_device(n, 5, np.uint64)
            part, keep = P.make_partitioning(fixed_len=L)
            cap = P.leco_max_blob_bytes(n, P.LECO_U64, part)
            size = torch.zeros(1, dtype=torch.uint64, device="cuda")
            row, blobs = {"L": L, "n": n}, []
            for name, c in (("default", auto), ("two_pass", two)):
                buf = torch.empty(cap, dtype=torch.uint8, device="cuda")
                f = lambda: c.check("leco_encode_async", P.leco_encode_async(
                    c.ctx, d, n, P.LECO_U64, part, buf, cap, size))
                f()
                c.sync()
                blobs.append(buf[: int(size.item())].clone())
                reps = max(5, min(200, int(2e9 / n)))
                row[f"{name}_us"] = round(time_stream(torch, stream, f, reps) * 1e6, 2)
            assert torch.equal(blobs[0], blobs[1]), f"encode_latency: blobs differ at L {L} n {n}"
            log(f"encode latency: {row}")
            rows.append(row)
            del d, blobs, keep
    torch.cuda.empty_cache()
    head = next(r for r in rows if r["L"] == 1024 and r["n"] == 10**6)
    res = {
        "metric": "decoded GB/s + lookups/s vs HBM roofline (batched/served vs plain); p99 latency",
        "value": head["default_us"], "unit": "us per encode (1e6 uint64 values, partitions of 1024)",
        "n_gpus": 1, "steps": None, "warmup": 1, "ms_per_step": round(head["default_us"] / 1e3, 5),
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "u64",
        "data": "synthetic (seeded lognormal-gap sorted keys)",
        "config": {"workload": "encode latency: one uint64 column of 1e4..1e8 values, partitions "
                               "of 1024 and 4096, default context against two passes"},
        "sizes": rows,
        "roofline": None,
        "cpu_baseline": None,
    }
    print(json.dumps(res), flush=True)
    auto.close()
    two.close()


def bench_higher_order(args):
    """The polynomial regressor on the evaluation's higher-order data: a
    two-sine signal with Gaussian noise (1e8 uint32 values, partitions of
    1000) and blocks of random cubics (2e8 uint64 values, partitions of
    2000).  Sizes, encode and decode times against the least-squares line."""
    import torch
    import paper_2306_15374_amd as P
    from paper_2306_15374_amd import workloads as W

    codec = P.Codec(0)
    stream = torch.cuda.current_stream()
    cols = {}
    t_dec_all = out_all = alg_all = 0.0
    for name, gen, n, L in (("cosmos", W.cosmos, 100_000_000, 1000),
                            ("poly_blocks", W.poly_blocks, 200_000_000, 2000)):
        log(f"{name}: drawing {n} values")
        col = gen(n, 71)
        d = torch.from_numpy(col).cuda()
        w = col.dtype.itemsize
        dt = P.LECO_U32 if w == 4 else P.LECO_U64
        res = {"n": n, "dtype": col.dtype.name, "L": L}
        pos = torch.from_numpy(W.uniform_positions(n, 10_000_000, 81)).cuda()
        for reg in ("ls", "poly"):
            part, _ = P.make_partitioning(fixed_len=L, regressor=reg)
            cap = P.leco_max_blob_bytes(n, dt, part)
            buf = torch.empty(cap, dtype=torch.uint8, device="cuda")
            size = torch.zeros(1, dtype=torch.uint64, device="cuda")
            enc = lambda: codec.check("leco_encode_async", P.leco_encode_async(
                codec.ctx, d, n, dt, part, buf, cap, size))
            enc()
            codec.sync()
            t_enc = time_events(torch, stream, enc, 3)
            codec.sync()
            nbytes = int(size.item())
            blob = buf[:nbytes]
            out = torch.empty_like(d)
            dec = lambda: codec.check("leco_decode_all", P.leco_decode_all(
                codec.ctx, blob, nbytes, out, n))
            dec()
            codec.sync()
            assert torch.equal(out, d), f"{name} {reg}: round trip"
            t_dec = time_stream(torch, stream, dec, max(3, min(args.steps, 10)))
            t_dec_iso = time_events(torch, stream, dec, max(3, min(args.steps, 10)))
            ra_out = torch.empty(pos.numel(), dtype=d.dtype, device="cuda")
            ra = lambda: codec.check("leco_random_access", P.leco_random_access(
                codec.ctx, blob, nbytes, pos, pos.numel(), ra_out))
            ra()
            codec.sync()
            t_ra = time_events(torch, stream, ra, 3)
            codec.sync()
            res[reg] = {"blob_bytes": nbytes, "ratio": round(nbytes / (w * n), 5),
                        "encode_ms": round(t_enc * 1e3, 3), "decode_all_ms": round(t_dec * 1e3, 4),
                        "decode_all_ms_isolated": round(t_dec_iso * 1e3, 4),
                        "decode_GBps": round(w * n / t_dec / 1e9, 1),
                        "decode_hbm_frac": round((nbytes + w * n) / t_dec / HBM_PEAK, 4),
                        "lookups_per_s": round(pos.numel() / t_ra, 1)}
            if reg == "poly":
                t_dec_all += t_dec
                out_all += w * n
                alg_all += nbytes + w * n
            del buf, blob, out
        res["poly_smaller_pct"] = round(100 * (res["ls"]["blob_bytes"] - res["poly"]["blob_bytes"])
                                        / res["ls"]["blob_bytes"], 2)
        log(f"{name}: {res}")
        cols[name] = res
        del d, pos
        torch.cuda.empty_cache()
    res = {
        "metric": "decoded GB/s + lookups/s vs HBM roofline (batched/served vs plain); p99 latency",
        "value": round(out_all / t_dec_all / 1e9, 2), "unit": "GB/s decoded (decode_all, polynomial blobs)",
        "n_gpus": 1, "steps": args.steps, "warmup": 1, "ms_per_step": round(t_dec_all * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32/u64",
        "data": "synthetic (seeded two-sine signal with Gaussian noise; blocks of random cubics)",
        "config": {"workload": "polynomial regressor: 1e8 uint32 two-sine values (L 1000) and "
                               "2e8 uint64 cubic-block values (L 2000)"},
        "columns": cols,
        "roofline": {"bound": "hbm", "achieved": round(alg_all / t_dec_all / 1e9, 1),
                     "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                     "frac": round(alg_all / t_dec_all / HBM_PEAK, 4), "traffic": None,
                     "kernel": "k_decode (polynomial path)", "bytes_per_launch": None},
        "cpu_baseline": None,
    }
    print(json.dumps(res), flush=True)
    codec.close()


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}): the codec has "
              "no multi-GPU path.", file=sys.stderr)
        sys.exit(2)
    if args.workload == "batched":
        print(json.dumps(bench_batched(args)), flush=True)
        return
    if args.workload == "served":
        print(json.dumps(bench_served(args)), flush=True)
        return
    if args.workload == "variable":
        return bench_variable(args)
    if args.workload == "encode_options":
        return bench_encode_options(args)
    if args.workload == "higher_order":
        return bench_higher_order(args)
    if args.workload == "encode_latency":
        return bench_encode_latency(args)
    import torch
    import paper_2306_15374_amd as P
    from paper_2306_15374_amd import workloads as W

    L = W.C2_L
    log(f"generating {args.n} keys and {args.lookups} positions")
    col = W.lognormal_keys(args.n, W.C2_SEED)
    pos = W.uniform_positions(args.n, args.lookups, W.C2_RA_SEED)
    codec = P.Codec(0)
    stream = torch.cuda.current_stream()
    d_col = torch.from_numpy(col).cuda()
    d_pos = torch.from_numpy(pos).cuda()
    torch.cuda.synchronize()

    log("encoding on the GPU")
    t0 = time.perf_counter()
    blob = codec.encode(d_col, fixed_len=L)
    torch.cuda.synchronize()
    t_enc_first = time.perf_counter() - t0
    # timed re-encode into the same buffer (scratch already allocated)
    part, _ = P.make_partitioning(fixed_len=L)
    cap = P.leco_max_blob_bytes(args.n, P.LECO_U64, part)
    buf = torch.empty(cap, dtype=torch.uint8, device="cuda")
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    st, size = P.leco_encode(codec.ctx, d_col, args.n, P.LECO_U64, part, buf, cap)
    e1.record(stream)
    codec.check("leco_encode", st)
    torch.cuda.synchronize()
    t_enc = e0.elapsed_time(e1) / 1e3
    blob_bytes = blob.numel()
    assert size == blob_bytes and torch.equal(buf[:size], blob)
    ratio = blob_bytes / (args.n * 8)
    log(f"blob {blob_bytes} bytes, ratio {ratio:.4f}, encode {t_enc * 1e3:.2f} ms")

    out = torch.empty(args.n, dtype=torch.uint64, device="cuda")
    ra_out = torch.empty(args.lookups, dtype=torch.uint64, device="cuda")

    def step(ev=None):
        if ev is not None:
            ev[0].record(stream)
        codec.check("leco_decode_all", P.leco_decode_all(codec.ctx, blob, blob_bytes, out, args.n))
        if ev is not None:
            ev[1].record(stream)
        codec.check("leco_random_access", P.leco_random_access(codec.ctx, blob, blob_bytes, d_pos,
                                                               args.lookups, ra_out))
        if ev is not None:
            ev[2].record(stream)

    log("parity at full size")
    step()
    codec.sync()
    assert torch.equal(out.view(torch.int64), d_col.view(torch.int64)), "decode_all != input"
    assert torch.equal(ra_out.view(torch.int64), d_col.view(torch.int64)[d_pos.view(torch.int64)]), \
        "random_access != input[pos]"

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(evs[k])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    codec.sync()
    t_dec = np.mean([e[0].elapsed_time(e[1]) for e in evs]) / 1e3
    t_ra = np.mean([e[1].elapsed_time(e[2]) for e in evs]) / 1e3
    out_bytes = args.n * 8
    dec_gbps = out_bytes / t_dec / 1e9
    alg_bytes = blob_bytes + out_bytes
    lookups = args.lookups / t_ra
    ra_alg = args.lookups * (8 + 8 + 8)        # position, output, residual word
    ra_gran = args.lookups * (8 + 8 + 64)      # residual touch at 64-byte granularity
    log(f"decode_all {t_dec * 1e3:.3f} ms = {dec_gbps:.1f} GB/s decoded, "
        f"{alg_bytes / t_dec / 1e9:.1f} GB/s algorithmic; random_access {t_ra * 1e3:.2f} ms = "
        f"{lookups:.3e} lookups/s")

    # HBM reference: the library's plain streaming copy and fill kernels over
    # the same 1.6 GB buffers (also the known-size kernel for the traffic
    # counters), and the runtime's own device-to-device copy of them.
    cal = {}
    out_u8, col_u8 = out.view(torch.uint8), d_col.view(torch.uint8)
    for name, fn, moved in (
            ("copy", lambda: codec.check("leco_diag_copy", P.leco_diag_copy(
                codec.ctx, d_col, out, out_bytes)), 2 * out_bytes),
            ("fill", lambda: codec.check("leco_diag_copy", P.leco_diag_copy(
                codec.ctx, None, out, out_bytes)), out_bytes),
            ("runtime_d2d_copy", lambda: out_u8.copy_(col_u8), 2 * out_bytes)):
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(5):
            c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            c0.record(stream)
            fn()
            c1.record(stream)
            torch.cuda.synchronize()
            ts.append(c0.elapsed_time(c1) / 1e3)
        cal[f"{name}_GBps"] = round(moved / float(np.median(ts)) / 1e9, 1)
    log(f"HBM reference: {cal}")

    cpu = None
    if not args.no_cpu_baseline:
        log("timing the CPU oracle")
        cpu = cpu_baseline(col, pos, args.cpu_sample, L, blob.cpu().numpy())

    res = {
        "metric": "decoded GB/s + lookups/s vs HBM roofline (batched/served vs plain); p99 latency",
        "value": round(dec_gbps, 2),
        "unit": "GB/s decoded (decode_all output)",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u64", "data": "synthetic (seeded lognormal-gap sorted keys)",
        "config": {"workload": "sorted uint64 keys, 200M values, partitions of 4096, "
                               "decode_all + 100M uniform random_access",
                   "n": args.n, "partition_len": L, "lookups": args.lookups},
        "lookups_per_s": round(lookups, 1),
        "random_access_ms": round(t_ra * 1e3, 4),
        "random_access_hbm_frac": {"algorithmic_24B": round(ra_alg / t_ra / HBM_PEAK, 4),
                                   "granular_80B": round(ra_gran / t_ra / HBM_PEAK, 4)},
        "decode_all_ms": round(t_dec * 1e3, 4),
        "compression_ratio": round(ratio, 5),
        "encode_GBps": round(out_bytes / t_enc / 1e9, 2),
        # the column read once and the blob written, against 8 TB/s
        "encode_hbm_frac": round((out_bytes + blob_bytes) / t_enc / HBM_PEAK, 4),
        "roofline": {"bound": "hbm", "achieved": round(alg_bytes / t_dec / 1e9, 1),
                     "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                     "frac": round(alg_bytes / t_dec / HBM_PEAK, 4),
                     "traffic": measured_traffic() if args.n == 200_000_000 else None,
                     "kernel": "k_decode", "bytes_per_launch": alg_bytes,
                     "frac_of_measured_copy": round(alg_bytes / t_dec / 1e9 / cal["copy_GBps"], 4)},
        "hbm_reference": cal,
        "cpu_baseline": cpu,
    }
    if not args.c2_only:
        # the other two workloads of the same run, on the freed device
        del out, ra_out, d_col, d_pos, blob, buf, out_u8, col_u8
        del col, pos
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        res["batched"] = strip(bench_batched(args, codec))
        res["served"] = strip(bench_served(args, codec))
    print(json.dumps(res), flush=True)
    codec.close()


def strip(res: dict) -> dict:
    """A workload's result without the keys the headline line already has."""
    drop = {"metric", "n_gpus", "steps", "warmup", "higher_is_better", "scaling", "vs_baseline",
            "cpu_baseline", "data"}
    return {k: v for k, v in res.items() if k not in drop}


if __name__ == "__main__":
    main()
