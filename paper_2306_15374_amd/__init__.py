"""MI355X-native LeCo codec: Python binding of ``libleco_hip.so``.

Argument marshalling only: every step of encoding and decoding runs in the
HIP kernels of the library (see ``include/leco.h`` for the C ABI and the
blob format).  PyTorch supplies device memory and streams.  There is no CPU
fallback: if the library is missing, every call raises.

Low-level functions carry the C names (``leco_encode``, ``leco_decode_all``,
...), take a context, torch CUDA tensors and a stream, and return the
status.  ``Codec`` wraps them for convenience.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libleco_hip.so")

LECO_OK, LECO_EINVAL, LECO_ENOMEM, LECO_ENOSPC, LECO_EFORMAT, LECO_ERANGE, LECO_EDEVICE = range(7)
LECO_U32, LECO_U64 = 4, 8
LECO_NOALLOC_SCRATCH_BYTES = 32 << 20
STATUS_NAMES = {0: "LECO_OK", 1: "LECO_EINVAL", 2: "LECO_ENOMEM", 3: "LECO_ENOSPC",
                4: "LECO_EFORMAT", 5: "LECO_ERANGE", 6: "LECO_EDEVICE"}

# Every symbol include/leco.h declares (checked by the ABI tests).
EXPORTS = [
    "leco_create", "leco_destroy", "leco_last_error", "leco_sync", "leco_max_blob_bytes",
    "leco_blob_info", "leco_validate_blob", "leco_encode", "leco_encode_async",
    "leco_encode_noalloc",
    "leco_decode_all", "leco_decode_range", "leco_random_access", "leco_filter_sum",
    "leco_diag_slope", "leco_diag_copy", "leco_encode_batch", "leco_batch_create",
    "leco_batch_destroy", "leco_batch_run", "leco_batch_run_graph", "leco_batch_tune",
    "leco_batch_tune_cached",
    "leco_batch_set_shape", "leco_server_start", "leco_server_submit", "leco_server_submit_batch",
    "leco_server_poll", "leco_server_release", "leco_server_stats_get", "leco_server_stop",
    "leco_server_replay", "leco_server_stats_reset", "leco_plain_replay", "leco_partition",
    "leco_fixed_cost", "leco_size_search",
]
LECO_REQ_RANDOM_ACCESS, LECO_REQ_RANGE, LECO_REQ_RANDOM_ACCESS_DEV = 1, 2, 3
LECO_BATCH_DECODE, LECO_BATCH_FILTER = 1, 2


class LecoError(RuntimeError):
    def __init__(self, fn: str, status: int, detail: str = ""):
        super().__init__(f"{fn}: {STATUS_NAMES.get(status, status)} {detail}".strip())
        self.status = status


class PartitionParams(C.Structure):
    _fields_ = [("tau", C.c_double), ("sm_bits", C.c_uint64), ("max_len", C.c_uint64),
                ("max_passes", C.c_uint64), ("start_positions", C.c_int32),
                ("reserved", C.c_int32)]


class EncodeJob(C.Structure):
    _fields_ = [("col_dev", C.c_void_p), ("n", C.c_uint64), ("dtype", C.c_int),
                ("force_constant_model", C.c_int32), ("fixed_len", C.c_uint64),
                ("blob_dev", C.c_void_p), ("blob_cap", C.c_uint64),
                ("blob_bytes_dev", C.c_void_p), ("regressor", C.c_int32),
                ("reserved", C.c_int32)]


class DecodeJob(C.Structure):
    _fields_ = [("blob_dev", C.c_void_p), ("blob_bytes", C.c_uint64), ("n", C.c_uint64),
                ("out_dev", C.c_void_p), ("lo", C.c_uint64), ("hi", C.c_uint64),
                ("sum3_dev", C.c_void_p)]


class ResidentCol(C.Structure):
    _fields_ = [("blob_dev", C.c_void_p), ("blob_bytes", C.c_uint64), ("n", C.c_uint64)]


class ServerConfig(C.Structure):
    _fields_ = [("out_budget_bytes", C.c_uint64), ("max_inflight", C.c_uint32),
                ("num_streams", C.c_uint32), ("max_step_items", C.c_uint32),
                ("max_step_positions", C.c_uint32), ("min_step_bytes", C.c_uint64),
                ("max_wait_us", C.c_uint32), ("reserved", C.c_uint32),
                ("position_ring_bytes", C.c_uint64)]


class Request(C.Structure):
    _fields_ = [("kind", C.c_uint32), ("col", C.c_uint32), ("positions", C.c_void_p),
                ("k", C.c_uint64), ("begin", C.c_uint64), ("end", C.c_uint64)]


class Completion(C.Structure):
    _fields_ = [("ticket", C.c_uint64), ("status", C.c_int32), ("dtype", C.c_int32),
                ("out_dev", C.c_void_p), ("count", C.c_uint64), ("latency_us", C.c_double)]


class ServerStats(C.Structure):
    _fields_ = [(name, C.c_uint64) for name in
                ("submitted", "completed", "steps", "values_out", "positions",
                 "out_bytes_in_use", "out_bytes_peak", "queued", "items",
                 "host_submit_ns", "host_admit_ns", "host_build_ns", "host_launch_ns",
                 "host_retire_ns", "host_wait_ns", "gpu_step_ns", "gpu_busy_ns", "gpu_span_ns")]


class Partitioning(C.Structure):
    _fields_ = [("fixed_len", C.c_uint64), ("starts_host", C.c_void_p),
                ("num_partitions", C.c_uint64), ("force_constant_model", C.c_int32),
                ("regressor", C.c_int32)]


_lib = None


def lib() -> C.CDLL:
    """Loads the HIP library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2306_15374_amd.build`")
        _lib = _bind(C.CDLL(LIB_PATH))
    return _lib


def _bind(L: C.CDLL) -> C.CDLL:
    u64, vp, i32 = C.c_uint64, C.c_void_p, C.c_int
    P = C.POINTER
    sig = {
        "leco_create": ([i32, P(vp)], i32),
        "leco_destroy": ([vp], i32),
        "leco_last_error": ([vp], C.c_char_p),
        "leco_sync": ([vp, vp], i32),
        "leco_max_blob_bytes": ([u64, i32, P(Partitioning), P(u64)], i32),
        "leco_blob_info": ([vp, P(u64), P(i32), P(u64)], i32),
        "leco_validate_blob": ([vp, vp, u64, vp], i32),
        "leco_encode": ([vp, vp, u64, i32, P(Partitioning), vp, u64, P(u64), vp], i32),
        "leco_encode_async": ([vp, vp, u64, i32, P(Partitioning), vp, u64, vp, vp], i32),
        "leco_encode_noalloc": ([vp, vp, u64, i32, P(Partitioning), vp, u64, vp, vp], i32),
        "leco_decode_all": ([vp, vp, u64, vp, u64, vp], i32),
        "leco_decode_range": ([vp, vp, u64, u64, u64, vp, vp], i32),
        "leco_random_access": ([vp, vp, u64, vp, u64, vp, vp], i32),
        "leco_filter_sum": ([vp, vp, u64, u64, u64, vp, vp], i32),
        "leco_diag_slope": ([vp, vp, u64, vp, vp], i32),
        "leco_diag_copy": ([vp, vp, vp, u64, vp], i32),
        "leco_encode_batch": ([vp, vp, u64, vp], i32),
        "leco_batch_create": ([vp, vp, u64, P(vp)], i32),
        "leco_batch_destroy": ([vp], i32),
        "leco_batch_run": ([vp, i32, vp], i32),
        "leco_batch_run_graph": ([vp, i32, vp], i32),
        "leco_batch_tune": ([vp, i32, vp, P(C.c_uint32), P(C.c_uint32)], i32),
        "leco_batch_tune_cached": ([vp, i32, C.c_char_p, vp, P(C.c_uint32), P(C.c_uint32), P(C.c_int32)], i32),
        "leco_batch_set_shape": ([vp, C.c_uint32, C.c_uint32], i32),
        "leco_server_start": ([vp, vp, u64, P(ServerConfig), P(vp)], i32),
        "leco_server_submit": ([vp, P(Request), P(u64)], i32),
        "leco_server_submit_batch": ([vp, P(Request), u64, P(u64), P(u64)], i32),
        "leco_server_poll": ([vp, vp, u64, P(u64)], i32),
        "leco_server_release": ([vp, u64], i32),
        "leco_server_stats_get": ([vp, P(ServerStats)], i32),
        "leco_server_stop": ([vp], i32),
        "leco_server_replay": ([vp, vp, vp, u64, vp, P(C.c_double)], i32),
        "leco_server_stats_reset": ([vp], i32),
        "leco_plain_replay": ([vp, vp, u64, vp, vp, u64, vp, u64, vp, vp, P(C.c_double)], i32),
        "leco_partition": ([vp, vp, u64, i32, P(PartitionParams), vp, u64, P(u64), vp], i32),
        "leco_fixed_cost": ([vp, vp, u64, i32, vp, u64, u64, u64, i32, P(u64), vp], i32),
        "leco_size_search": ([vp, vp, u64, i32, vp, u64, u64, i32, P(u64), P(u64), vp, u64,
                              P(u64), vp], i32),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    return L


def _stream(stream) -> int:
    import torch
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)


def _ptr(t) -> int | None:
    """Device or host address of a tensor, or an address given as an int."""
    if t is None or isinstance(t, int):
        return t
    return t.data_ptr()


def _dtype_code(t) -> int:
    import torch
    if t.dtype in (torch.uint32, torch.int32):
        return LECO_U32
    if t.dtype in (torch.uint64, torch.int64):
        return LECO_U64
    raise TypeError(f"column dtype must be 32- or 64-bit integer, got {t.dtype}")


REGRESSORS = {"ls": 0, "minimax": 1, "poly": 2}  # leco_regressor


def regressor_code(name: str) -> int:
    try:
        return REGRESSORS[name]
    except KeyError:
        raise ValueError(f"regressor must be one of {sorted(REGRESSORS)}, got {name!r}") from None


def make_partitioning(fixed_len: int = 0, starts=None, force_constant: bool = False,
                      regressor: str = "ls"):
    """Returns (Partitioning, keepalive) for a fixed length or host starts."""
    import numpy as np
    reg = regressor_code(regressor)
    if fixed_len:
        return Partitioning(fixed_len, None, 0, int(force_constant), reg), None
    s = np.ascontiguousarray(starts, dtype=np.uint64)
    return Partitioning(0, s.ctypes.data, len(s) - 1, int(force_constant), reg), s


# ---- C-named wrappers ----------------------------------------------------------

def leco_create(device: int = 0) -> int:
    h = C.c_void_p()
    st = lib().leco_create(device, C.byref(h))
    if st != LECO_OK:
        raise LecoError("leco_create", st)
    return h.value


def leco_destroy(ctx: int) -> int:
    return lib().leco_destroy(ctx)


def leco_last_error(ctx: int) -> str:
    return (lib().leco_last_error(ctx) or b"").decode()


def leco_sync(ctx: int, stream=None) -> int:
    return lib().leco_sync(ctx, _stream(stream))


def leco_max_blob_bytes(n: int, dtype: int, part: Partitioning) -> int:
    out = C.c_uint64()
    st = lib().leco_max_blob_bytes(n, dtype, C.byref(part), C.byref(out))
    if st != LECO_OK:
        raise LecoError("leco_max_blob_bytes", st)
    return out.value


def leco_blob_info(header_bytes: bytes):
    buf = C.create_string_buffer(bytes(header_bytes[:64]), 64)
    n, dt, m = C.c_uint64(), C.c_int(), C.c_uint64()
    st = lib().leco_blob_info(buf, C.byref(n), C.byref(dt), C.byref(m))
    if st != LECO_OK:
        raise LecoError("leco_blob_info", st)
    return n.value, dt.value, m.value


def leco_validate_blob(ctx: int, blob, blob_bytes: int, stream=None) -> int:
    return lib().leco_validate_blob(ctx, _ptr(blob), blob_bytes, _stream(stream))


def leco_encode(ctx: int, col, n: int, dtype: int, part: Partitioning, blob, blob_cap: int,
                stream=None) -> tuple[int, int]:
    size = C.c_uint64()
    st = lib().leco_encode(ctx, _ptr(col), n, dtype, C.byref(part), _ptr(blob), blob_cap,
                           C.byref(size), _stream(stream))
    return st, size.value


def leco_encode_async(ctx: int, col, n: int, dtype: int, part: Partitioning, blob,
                      blob_cap: int, size_dev, stream=None) -> int:
    return lib().leco_encode_async(ctx, _ptr(col), n, dtype, C.byref(part), _ptr(blob),
                                   blob_cap, _ptr(size_dev), _stream(stream))


def leco_encode_noalloc(ctx: int, col, n: int, dtype: int, part: Partitioning, blob,
                        blob_cap: int, size_dev, stream=None) -> int:
    return lib().leco_encode_noalloc(ctx, _ptr(col), n, dtype, C.byref(part), _ptr(blob),
                                     blob_cap, _ptr(size_dev), _stream(stream))


def leco_decode_all(ctx: int, blob, blob_bytes: int, out, out_cap: int, stream=None) -> int:
    return lib().leco_decode_all(ctx, _ptr(blob), blob_bytes, _ptr(out), out_cap, _stream(stream))


def leco_decode_range(ctx: int, blob, blob_bytes: int, begin: int, end: int, out,
                      stream=None) -> int:
    return lib().leco_decode_range(ctx, _ptr(blob), blob_bytes, begin, end, _ptr(out),
                                   _stream(stream))


def leco_random_access(ctx: int, blob, blob_bytes: int, pos, k: int, out, stream=None) -> int:
    return lib().leco_random_access(ctx, _ptr(blob), blob_bytes, _ptr(pos), k, _ptr(out),
                                    _stream(stream))


def leco_filter_sum(ctx: int, blob, blob_bytes: int, lo: int, hi: int, out3, stream=None) -> int:
    return lib().leco_filter_sum(ctx, _ptr(blob), blob_bytes, lo, hi, _ptr(out3),
                                 _stream(stream))


def leco_diag_slope(ctx: int, pairs, k: int, out, stream=None) -> int:
    return lib().leco_diag_slope(ctx, _ptr(pairs), k, _ptr(out), _stream(stream))


def leco_diag_copy(ctx: int, src, dst, nbytes: int, stream=None) -> int:
    return lib().leco_diag_copy(ctx, _ptr(src), _ptr(dst), nbytes, _stream(stream))


def leco_encode_batch(ctx: int, jobs, stream=None) -> int:
    arr = (EncodeJob * len(jobs))(*jobs)
    return lib().leco_encode_batch(ctx, arr, len(jobs), _stream(stream))


def leco_batch_create(ctx: int, jobs) -> int:
    arr = (DecodeJob * len(jobs))(*jobs)
    h = C.c_void_p()
    st = lib().leco_batch_create(ctx, arr, len(jobs), C.byref(h))
    if st != LECO_OK:
        raise LecoError("leco_batch_create", st, leco_last_error(ctx))
    return h.value


def leco_batch_destroy(batch: int) -> int:
    return lib().leco_batch_destroy(batch)


def leco_batch_run(batch: int, op: int, stream=None) -> int:
    return lib().leco_batch_run(batch, op, _stream(stream))


def leco_batch_run_graph(batch: int, op: int, stream=None) -> int:
    return lib().leco_batch_run_graph(batch, op, _stream(stream))


def leco_batch_tune(batch: int, op: int, stream=None) -> tuple[int, int, int]:
    t, b = C.c_uint32(), C.c_uint32()
    st = lib().leco_batch_tune(batch, op, _stream(stream), C.byref(t), C.byref(b))
    return st, t.value, b.value


def leco_batch_tune_cached(batch: int, op: int, cache_path: str | None,
                           stream=None) -> tuple[int, int, int, bool]:
    """(status, tile_log2, blocks_per_cu, whether the shape came from the
    tuner cache file)."""
    t, b, hit = C.c_uint32(), C.c_uint32(), C.c_int32()
    path = None if cache_path is None else cache_path.encode()
    st = lib().leco_batch_tune_cached(batch, op, path, _stream(stream), C.byref(t), C.byref(b),
                                      C.byref(hit))
    return st, t.value, b.value, bool(hit.value)


def leco_batch_set_shape(batch: int, tile_log2: int, blocks_per_cu: int) -> int:
    return lib().leco_batch_set_shape(batch, tile_log2, blocks_per_cu)


def leco_server_start(ctx: int, cols, cfg: ServerConfig) -> int:
    arr = (ResidentCol * len(cols))(*cols)
    h = C.c_void_p()
    st = lib().leco_server_start(ctx, arr, len(cols), C.byref(cfg), C.byref(h))
    if st != LECO_OK:
        raise LecoError("leco_server_start", st, leco_last_error(ctx))
    return h.value


def leco_server_submit(server: int, req: Request) -> tuple[int, int]:
    t = C.c_uint64()
    st = lib().leco_server_submit(server, C.byref(req), C.byref(t))
    return st, t.value



def leco_server_submit_batch(server: int, reqs) -> tuple[int, list[int]]:
    """reqs: a ctypes Request array.  Returns (status, tickets of the
    accepted prefix)."""
    n = len(reqs)
    tickets = (C.c_uint64 * max(n, 1))()
    acc = C.c_uint64()
    st = lib().leco_server_submit_batch(server, reqs, n, tickets, C.byref(acc))
    return st, [int(tickets[i]) for i in range(acc.value)]

def leco_server_poll(server: int, max_n: int = 256) -> list:
    arr = (Completion * max_n)()
    got = C.c_uint64()
    st = lib().leco_server_poll(server, arr, max_n, C.byref(got))
    if st != LECO_OK:
        raise LecoError("leco_server_poll", st)
    return [arr[i] for i in range(got.value)]


def leco_server_release(server: int, ticket: int) -> int:
    return lib().leco_server_release(server, ticket)


def leco_server_stats_get(server: int) -> dict:
    s = ServerStats()
    st = lib().leco_server_stats_get(server, C.byref(s))
    if st != LECO_OK:
        raise LecoError("leco_server_stats_get", st)
    return {name: getattr(s, name) for name, _ in ServerStats._fields_}


def leco_server_stats_reset(server: int) -> int:
    return lib().leco_server_stats_reset(server)


def leco_plain_replay(ctx: int, cols, reqs, arrival_s, out, out_bytes: int, stream=None,
                      latencies_out=None) -> tuple[int, float]:
    """The plain one-launch-per-request path over the same request stream
    (reqs: a ctypes Request array of ranges and device-position lookups)."""
    arr = (ResidentCol * len(cols))(*cols)
    el = C.c_double()
    st = lib().leco_plain_replay(ctx, arr, len(cols), reqs, arrival_s.ctypes.data, len(arrival_s),
                                 _ptr(out), out_bytes, _stream(stream),
                                 None if latencies_out is None else latencies_out.ctypes.data,
                                 C.byref(el))
    return st, el.value


def leco_server_stop(server: int) -> int:
    return lib().leco_server_stop(server)


def leco_server_replay(server: int, reqs, arrival_s, latencies_out=None) -> tuple[int, float]:
    """reqs: a ctypes Request array; arrival_s and latencies_out: float64
    numpy arrays of the same length."""
    el = C.c_double()
    st = lib().leco_server_replay(server, reqs, arrival_s.ctypes.data, len(arrival_s),
                                  None if latencies_out is None else latencies_out.ctypes.data,
                                  C.byref(el))
    return st, el.value


def leco_partition(ctx: int, col, n: int, dtype: int, params: PartitionParams,
                   starts_out, stream=None) -> tuple[int, int]:
    """starts_out: a uint64 numpy array with room for m + 1 starts."""
    m = C.c_uint64()
    st = lib().leco_partition(ctx, _ptr(col), n, dtype, C.byref(params), starts_out.ctypes.data,
                              len(starts_out), C.byref(m), _stream(stream))
    return st, m.value


def leco_fixed_cost(ctx: int, col, n: int, dtype: int, starts, window: int, L: int,
                    regressor: int = 0, stream=None) -> tuple[int, int]:
    """starts: a uint64 numpy array of window starts (host)."""
    cost = C.c_uint64()
    st = lib().leco_fixed_cost(ctx, _ptr(col), n, dtype, starts.ctypes.data if len(starts) else None,
                               len(starts), window, L, regressor, C.byref(cost), _stream(stream))
    return st, cost.value


def leco_size_search(ctx: int, col, n: int, dtype: int, starts, window: int, regressor: int = 0,
                     trace_out=None, stream=None) -> tuple[int, int, int, int]:
    """Returns (status, L, cost, evaluations); trace_out (uint64 numpy array,
    optional) receives (L, cost) pairs."""
    L, cost, tl = C.c_uint64(), C.c_uint64(), C.c_uint64()
    st = lib().leco_size_search(ctx, _ptr(col), n, dtype,
                                starts.ctypes.data if len(starts) else None, len(starts), window,
                                regressor, C.byref(L), C.byref(cost),
                                None if trace_out is None else trace_out.ctypes.data,
                                0 if trace_out is None else len(trace_out), C.byref(tl),
                                _stream(stream))
    return st, L.value, cost.value, tl.value


# ---- convenience wrapper --------------------------------------------------------------

class Codec:
    """A context on one device plus tensor-level helpers.  Blobs are uint8
    CUDA tensors whose length is the blob size."""

    def __init__(self, device: int = 0):
        import torch
        self.device = torch.device("cuda", device)
        self.ctx = leco_create(device)

    def close(self):
        if self.ctx:
            leco_destroy(self.ctx)
            self.ctx = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def check(self, fn: str, st: int):
        if st != LECO_OK:
            raise LecoError(fn, st, leco_last_error(self.ctx))

    def sync(self, stream=None):
        self.check("leco_sync", leco_sync(self.ctx, stream))

    def encode(self, col, fixed_len: int = 0, starts=None, force_constant: bool = False,
               stream=None, regressor: str = "ls"):
        """Encodes a CUDA tensor column; returns the blob (uint8 tensor)."""
        import torch
        dt = _dtype_code(col)
        part, keep = make_partitioning(fixed_len, starts, force_constant, regressor)
        cap = leco_max_blob_bytes(col.numel(), dt, part)
        buf = torch.empty(cap, dtype=torch.uint8, device=col.device)
        st, size = leco_encode(self.ctx, col, col.numel(), dt, part, buf, cap, stream)
        del keep
        self.check("leco_encode", st)
        return buf[:size]

    def partition(self, col, tau: float = 0.1, sm_bits: int = 320, max_len: int = 1 << 20,
                  max_passes: int = 0, stream=None, start_positions: bool = False):
        """Variable-length partition starts of a CUDA tensor column (numpy
        uint64 array of m + 1 starts)."""
        import numpy as np
        params = PartitionParams(tau, sm_bits, max_len, max_passes, int(start_positions), 0)
        # room for a mean partition length down to 16; a finer result is
        # computed again with the exact size
        cap = max(1024, col.numel() // 16 + 2)
        while True:
            out = np.zeros(cap, dtype=np.uint64)
            st, m = leco_partition(self.ctx, col, col.numel(), _dtype_code(col), params, out, stream)
            if st == LECO_ENOSPC and m + 1 > cap:
                cap = m + 1
                continue
            self.check("leco_partition", st)
            return out[: m + 1].copy()

    def fixed_cost(self, col, starts, window: int, L: int, regressor: str = "ls", stream=None):
        """Sampled record + word bytes of fixed partitions of length L over
        the windows [starts[i], starts[i] + window)."""
        import numpy as np
        s = np.ascontiguousarray(starts, dtype=np.uint64)
        st, cost = leco_fixed_cost(self.ctx, col, col.numel(), _dtype_code(col), s, window, L,
                                   regressor_code(regressor), stream)
        self.check("leco_fixed_cost", st)
        return cost

    def size_search(self, col, starts, window: int, regressor: str = "ls", stream=None) -> dict:
        """Fixed partition length search over sampled windows (section
        3.2.1); returns {"L", "cost", "trace": [(L, cost), ...]}."""
        import numpy as np
        s = np.ascontiguousarray(starts, dtype=np.uint64)
        trace = np.zeros(2 * 4096, dtype=np.uint64)
        st, L, cost, n = leco_size_search(self.ctx, col, col.numel(), _dtype_code(col), s, window,
                                          regressor_code(regressor), trace, stream)
        self.check("leco_size_search", st)
        steps = [(int(trace[2 * i]), int(trace[2 * i + 1])) for i in range(min(n, len(trace) // 2))]
        return {"L": L, "cost": cost, "trace": steps}

    def info(self, blob):
        return leco_blob_info(bytes(blob[:64].cpu().numpy().tobytes()))

    def _out(self, n: int, dt: int, device):
        import torch
        return torch.empty(n, dtype=torch.uint32 if dt == LECO_U32 else torch.uint64, device=device)

    def decode_all(self, blob, out=None, stream=None, sync: bool = True):
        n, dt, _ = self.info(blob)
        if out is None:
            out = self._out(n, dt, blob.device)
        self.check("leco_decode_all", leco_decode_all(self.ctx, blob, blob.numel(), out,
                                                      out.numel(), stream))
        if sync:
            self.sync(stream)
        return out

    def decode_range(self, blob, begin: int, end: int, out=None, stream=None, sync: bool = True):
        _, dt, _ = self.info(blob)
        if out is None:
            out = self._out(max(end - begin, 0), dt, blob.device)
        self.check("leco_decode_range", leco_decode_range(self.ctx, blob, blob.numel(), begin,
                                                          end, out, stream))
        if sync:
            self.sync(stream)
        return out

    def random_access(self, blob, pos, out=None, stream=None, sync: bool = True):
        _, dt, _ = self.info(blob)
        if out is None:
            out = self._out(pos.numel(), dt, blob.device)
        self.check("leco_random_access", leco_random_access(self.ctx, blob, blob.numel(), pos,
                                                            pos.numel(), out, stream))
        if sync:
            self.sync(stream)
        return out

    def filter_sum(self, blob, lo: int, hi: int, stream=None) -> tuple[int, int]:
        import torch
        out3 = torch.empty(3, dtype=torch.uint64, device=blob.device)
        self.check("leco_filter_sum", leco_filter_sum(self.ctx, blob, blob.numel(), lo, hi,
                                                      out3, stream))
        self.sync(stream)
        v = [int(x) for x in out3.cpu().numpy()]
        return (v[1] << 64) | v[0], v[2]

    def validate(self, blob, stream=None) -> int:
        return leco_validate_blob(self.ctx, blob, blob.numel(), stream)
