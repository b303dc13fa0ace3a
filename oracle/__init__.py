"""LeCo CPU oracle: ctypes wrapper around ``libleco_oracle.so``.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  The product (the
HIP library and its Python binding) never imports, links or calls it.

The C library is a plain scalar implementation of the LeCo paper's encoder,
decoder and variable-length partitioner (see ``leco_oracle.c``); this module
only marshals numpy arrays into it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libleco_oracle.so")
SOURCES = [os.path.join(_HERE, "leco_oracle.c")]

# Scalar, no FMA contraction, no fast-math, no -march: every floating-point
# operation is one correctly rounded binary64 operation.
CFLAGS = ["-O2", "-std=gnu11", "-fPIC", "-shared", "-ffp-contract=off",
          "-fno-fast-math", "-Wall", "-Wextra"]

OK, EINVAL, ENOMEM, ENOSPC, EFORMAT, ERANGE = 0, 1, 2, 3, 4, 5


class OracleError(RuntimeError):
    def __init__(self, fn: str, status: int):
        super().__init__(f"{fn} failed with status {status}")
        self.status = status


def build(extra_flags: list[str] | None = None, out: str | None = None) -> str:
    """Compile the oracle with gcc; returns the path of the shared library."""
    out = out or LIB_PATH
    cmd = ["gcc", *CFLAGS, *(extra_flags or []), "-o", out, *SOURCES, "-lm"]
    subprocess.run(cmd, check=True)
    return out


class _Model(C.Structure):
    _fields_ = [
        ("vmin", C.c_uint64), ("vmax", C.c_uint64), ("b_for", C.c_uint64),
        ("fitted", C.c_int32), ("mode", C.c_int32),
        ("N_lo", C.c_uint64), ("N_hi", C.c_int64),
        ("D_lo", C.c_uint64), ("D_hi", C.c_uint64),
        ("theta1_ls", C.c_double), ("r_min", C.c_int64), ("r_max", C.c_int64),
        ("b_ls", C.c_uint64), ("theta1", C.c_double), ("base", C.c_uint64),
        ("bits", C.c_uint64),
        ("mm_fitted", C.c_int32), ("mm_pad", C.c_int32),
        ("mm_dy", C.c_int64), ("mm_dt", C.c_uint64), ("theta1_mm", C.c_double),
        ("r_min_mm", C.c_int64), ("r_max_mm", C.c_int64), ("b_mm", C.c_uint64),
        ("poly_fitted", C.c_int32), ("poly_degree", C.c_int32), ("pc", C.c_double * 3),
        ("b_p2", C.c_uint64), ("b_p3", C.c_uint64), ("stored_c", C.c_double * 3),
    ]


REGRESSORS = {"ls": 0, "minimax": 1, "poly": 2}


def _regressor(name: str) -> int:
    try:
        return REGRESSORS[name]
    except KeyError:
        raise ValueError(f"regressor must be one of {sorted(REGRESSORS)}, got {name!r}") from None


COST_FN = C.CFUNCTYPE(C.c_uint64, C.c_void_p, C.c_uint64)

_lib = None


def lib() -> C.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        _lib = _bind(C.CDLL(LIB_PATH))
    return _lib


def _bind(L: C.CDLL) -> C.CDLL:
    u64, vp, P = C.c_uint64, C.c_void_p, C.POINTER
    L.leco_ref_bitlen.argtypes = [u64]
    L.leco_ref_bitlen.restype = u64
    L.leco_ref_fit.argtypes = [vp, u64, C.c_int, C.c_int, P(_Model)]
    L.leco_ref_fit.restype = C.c_int
    L.leco_ref_minimax_slope.argtypes = [vp, u64, P(C.c_int64), P(u64)]
    L.leco_ref_minimax_slope.restype = C.c_int
    L.leco_ref_blob_bytes.argtypes = [vp, u64, C.c_int, u64, vp, u64, C.c_int, C.c_int, P(u64)]
    L.leco_ref_encode.argtypes = [vp, u64, C.c_int, u64, vp, u64, C.c_int, C.c_int, vp, u64,
                                  P(u64)]
    L.leco_ref_blob_info.argtypes = [vp, u64, P(u64), P(C.c_int), P(u64)]
    L.leco_ref_blob_record.argtypes = [vp, u64, u64, P(u64), P(C.c_double), P(u64),
                                       P(u64), P(u64), P(u64)]
    L.leco_ref_decode_all.argtypes = [vp, u64, vp, u64]
    L.leco_ref_decode_range.argtypes = [vp, u64, u64, u64, vp]
    L.leco_ref_random_access.argtypes = [vp, u64, vp, u64, vp]
    L.leco_ref_filter_sum.argtypes = [vp, u64, u64, u64, vp]
    L.leco_ref_split_cost.argtypes = [vp, u64, u64, C.c_int]
    L.leco_ref_split_cost.restype = C.c_int64
    L.leco_ref_delta_partition_bits.argtypes = [vp, u64, u64, u64]
    L.leco_ref_delta_partition_bits.restype = u64
    L.leco_ref_partition_cost_bytes.argtypes = [vp, u64, u64]
    L.leco_ref_partition_cost_bytes.restype = u64
    L.leco_ref_partition_greedy.argtypes = [vp, u64, C.c_int, C.c_double, u64, u64, u64,
                                            C.c_int, vp, P(u64)]
    L.leco_ref_partition_split.argtypes = [vp, u64, C.c_int, C.c_double, u64, u64, C.c_int, vp,
                                           P(u64)]
    L.leco_ref_start_positions.argtypes = [vp, u64, C.c_int, vp, vp, P(u64)]
    L.leco_ref_start_positions_delta.argtypes = [vp, u64, C.c_int, vp, P(u64)]
    L.leco_ref_delta_fix_bytes.argtypes = [vp, u64, C.c_int, u64, P(u64)]
    L.leco_ref_delta_fix_encode.argtypes = [vp, u64, C.c_int, u64, vp, u64, P(u64)]
    L.leco_ref_delta_fix_decode.argtypes = [vp, u64, vp, u64]
    L.leco_ref_partition_merge.argtypes = [vp, u64, C.c_int, vp, P(u64), u64, u64]
    L.leco_ref_partition_dp.argtypes = [vp, u64, C.c_int, u64, vp, P(u64), P(u64)]
    L.leco_ref_partition_bruteforce.argtypes = [vp, u64, C.c_int, u64, vp, P(u64), P(u64)]
    L.leco_ref_partitioning_cost.argtypes = [vp, u64, C.c_int, vp, u64, P(u64)]
    L.leco_ref_fixed_cost.argtypes = [vp, u64, C.c_int, vp, u64, u64, u64, C.c_int, P(u64)]
    L.leco_ref_size_search_fn.argtypes = [u64, COST_FN, vp, P(u64), P(u64), vp, u64, P(u64)]
    L.leco_ref_size_search.argtypes = [vp, u64, C.c_int, vp, u64, u64, C.c_int, P(u64), P(u64),
                                       vp, u64, P(u64)]
    for name in ("leco_ref_blob_bytes", "leco_ref_encode", "leco_ref_blob_info",
                 "leco_ref_blob_record", "leco_ref_decode_all", "leco_ref_decode_range",
                 "leco_ref_random_access", "leco_ref_filter_sum",
                 "leco_ref_partition_greedy", "leco_ref_partition_merge",
                 "leco_ref_partition_split", "leco_ref_start_positions",
                 "leco_ref_start_positions_delta", "leco_ref_delta_fix_bytes",
                 "leco_ref_delta_fix_encode", "leco_ref_delta_fix_decode",
                 "leco_ref_partition_dp", "leco_ref_partition_bruteforce",
                 "leco_ref_partitioning_cost", "leco_ref_fixed_cost",
                 "leco_ref_size_search_fn", "leco_ref_size_search"):
        getattr(L, name).restype = C.c_int
    return L


def _ptr(a: np.ndarray | None) -> int | None:
    return None if a is None else a.ctypes.data


def _check(fn: str, st: int) -> None:
    if st != OK:
        raise OracleError(fn, st)


def _dtype_code(col: np.ndarray) -> int:
    if col.dtype == np.uint32:
        return 4
    if col.dtype == np.uint64:
        return 8
    raise TypeError(f"column dtype must be uint32 or uint64, got {col.dtype}")


def _np_dtype(code: int):
    return np.uint32 if code == 4 else np.uint64


def _starts_arg(fixed_len: int, starts):
    if fixed_len and fixed_len > 0:
        return fixed_len, None, 0
    s = np.ascontiguousarray(starts, dtype=np.uint64)
    return 0, s, len(s) - 1


def bitlen(x: int) -> int:
    return int(lib().leco_ref_bitlen(x))


def fit(values, force_constant: bool = False, regressor: str = "ls") -> dict:
    v = np.ascontiguousarray(values, dtype=np.uint64)
    md = _Model()
    _check("leco_ref_fit", lib().leco_ref_fit(_ptr(v), len(v), int(force_constant),
                                              _regressor(regressor), C.byref(md)))
    d = {name: getattr(md, name) for name, _ in _Model._fields_}
    d["pc"], d["stored_c"] = list(md.pc), list(md.stored_c)
    d["N"] = (d["N_hi"] << 64) | d["N_lo"]
    d["D"] = (d["D_hi"] << 64) | d["D_lo"]
    return d


def minimax_slope(values) -> tuple[int, int]:
    """Exact minimax slope (dy, dt) of the points (t, values[t])."""
    v = np.ascontiguousarray(values, dtype=np.uint64)
    dy, dt = C.c_int64(), C.c_uint64()
    _check("leco_ref_minimax_slope",
           lib().leco_ref_minimax_slope(_ptr(v), len(v), C.byref(dy), C.byref(dt)))
    return dy.value, dt.value


def blob_bytes(col: np.ndarray, fixed_len: int = 0, starts=None,
               force_constant: bool = False, regressor: str = "ls") -> int:
    col = np.ascontiguousarray(col)
    fl, s, m = _starts_arg(fixed_len, starts)
    out = C.c_uint64()
    _check("leco_ref_blob_bytes", lib().leco_ref_blob_bytes(
        _ptr(col), len(col), _dtype_code(col), fl, _ptr(s), m, int(force_constant),
        _regressor(regressor), C.byref(out)))
    return out.value


def encode(col: np.ndarray, fixed_len: int = 0, starts=None,
           force_constant: bool = False, regressor: str = "ls") -> np.ndarray:
    """Encode a uint32/uint64 column; returns the blob as a uint8 array."""
    col = np.ascontiguousarray(col)
    fl, s, m = _starts_arg(fixed_len, starts)
    size = C.c_uint64()
    L = lib()
    reg = _regressor(regressor)
    st = L.leco_ref_encode(_ptr(col), len(col), _dtype_code(col), fl, _ptr(s), m,
                           int(force_constant), reg, None, 0, C.byref(size))
    if st != ENOSPC:
        _check("leco_ref_encode", st)
    blob = np.zeros(size.value, dtype=np.uint8)
    _check("leco_ref_encode", L.leco_ref_encode(
        _ptr(col), len(col), _dtype_code(col), fl, _ptr(s), m, int(force_constant), reg,
        _ptr(blob), len(blob), C.byref(size)))
    return blob


def blob_info(blob: np.ndarray) -> tuple[int, int, int]:
    n, dt, m = C.c_uint64(), C.c_int(), C.c_uint64()
    _check("leco_ref_blob_info", lib().leco_ref_blob_info(
        _ptr(blob), len(blob), C.byref(n), C.byref(dt), C.byref(m)))
    return n.value, dt.value, m.value


def blob_record(blob: np.ndarray, j: int) -> dict:
    base, th, wo, bits, st, ln = (C.c_uint64(), C.c_double(), C.c_uint64(),
                                  C.c_uint64(), C.c_uint64(), C.c_uint64())
    _check("leco_ref_blob_record", lib().leco_ref_blob_record(
        _ptr(blob), len(blob), j, C.byref(base), C.byref(th), C.byref(wo),
        C.byref(bits), C.byref(st), C.byref(ln)))
    return dict(base=base.value, theta1=th.value, word_off=wo.value, bits=bits.value,
                start=st.value, len=ln.value)


def decode_all(blob: np.ndarray) -> np.ndarray:
    n, dt, _ = blob_info(blob)
    out = np.zeros(n, dtype=_np_dtype(dt))
    _check("leco_ref_decode_all", lib().leco_ref_decode_all(_ptr(blob), len(blob), _ptr(out), n))
    return out


def decode_range(blob: np.ndarray, begin: int, end: int) -> np.ndarray:
    n, dt, _ = blob_info(blob)
    out = np.zeros(max(end - begin, 0), dtype=_np_dtype(dt))
    _check("leco_ref_decode_range", lib().leco_ref_decode_range(
        _ptr(blob), len(blob), begin, end, _ptr(out)))
    return out


def random_access(blob: np.ndarray, positions) -> np.ndarray:
    n, dt, _ = blob_info(blob)
    pos = np.ascontiguousarray(positions, dtype=np.uint64)
    out = np.zeros(len(pos), dtype=_np_dtype(dt))
    _check("leco_ref_random_access", lib().leco_ref_random_access(
        _ptr(blob), len(blob), _ptr(pos), len(pos), _ptr(out)))
    return out


def filter_sum(blob: np.ndarray, lo: int, hi: int) -> tuple[int, int]:
    """Returns (exact sum, count) of decoded values v with lo <= v < hi."""
    out = np.zeros(3, dtype=np.uint64)
    _check("leco_ref_filter_sum", lib().leco_ref_filter_sum(
        _ptr(blob), len(blob), lo, hi, _ptr(out)))
    return (int(out[1]) << 64) | int(out[0]), int(out[2])


def split_cost(values, i: int, j: int, model: str = "linear") -> int:
    v = np.ascontiguousarray(values, dtype=np.uint64)
    return int(lib().leco_ref_split_cost(_ptr(v), i, j, 1 if model == "delta" else 0))


def delta_partition_bits(values, i: int, j: int, sm_bits: int) -> int:
    v = np.ascontiguousarray(values, dtype=np.uint64)
    return int(lib().leco_ref_delta_partition_bits(_ptr(v), i, j, sm_bits))


def partition_cost_bytes(values, i: int, j: int) -> int:
    v = np.ascontiguousarray(values, dtype=np.uint64)
    return int(lib().leco_ref_partition_cost_bytes(_ptr(v), i, j))


def partition_greedy(col: np.ndarray, tau: float = 0.1, sm_bits: int = 320,
                     max_len: int = 1 << 20, max_passes: int = 0,
                     start_positions: bool = False) -> np.ndarray:
    """Greedy split + merge scan (section 3.2.2); the partition starts."""
    col = np.ascontiguousarray(col)
    starts = np.zeros(len(col) + 1, dtype=np.uint64)
    m = C.c_uint64()
    _check("leco_ref_partition_greedy", lib().leco_ref_partition_greedy(
        _ptr(col), len(col), _dtype_code(col), tau, sm_bits, max_len, max_passes,
        int(start_positions), _ptr(starts), C.byref(m)))
    return starts[: m.value + 1].copy()


def partition_split(col: np.ndarray, tau: float = 0.1, sm_bits: int = 320,
                    max_len: int = 1 << 20, start_positions: bool = False) -> np.ndarray:
    """The split phase alone (section 3.2.2)."""
    col = np.ascontiguousarray(col)
    starts = np.zeros(len(col) + 1, dtype=np.uint64)
    m = C.c_uint64()
    _check("leco_ref_partition_split", lib().leco_ref_partition_split(
        _ptr(col), len(col), _dtype_code(col), tau, sm_bits, max_len, int(start_positions),
        _ptr(starts), C.byref(m)))
    return starts[: m.value + 1].copy()


def starting_partitions(col: np.ndarray) -> list[tuple[int, int]]:
    """Starting partitions of the linear regressor (section 3.2.2) as
    half-open [first, end) value ranges."""
    col = np.ascontiguousarray(col)
    first = np.zeros(max(len(col), 1), dtype=np.uint64)
    end = np.zeros(max(len(col), 1), dtype=np.uint64)
    c = C.c_uint64()
    _check("leco_ref_start_positions", lib().leco_ref_start_positions(
        _ptr(col), len(col), _dtype_code(col), _ptr(first), _ptr(end), C.byref(c)))
    return [(int(a), int(b)) for a, b in zip(first[: c.value], end[: c.value])]


def start_positions(col: np.ndarray) -> np.ndarray:
    """First values of the linear regressor's starting partitions."""
    return np.array([a for a, _ in starting_partitions(col)], dtype=np.uint64)


def start_positions_delta(col: np.ndarray) -> np.ndarray:
    """First values of Delta encoding's starting partitions (section 3.2.2,
    required bits and delta bits)."""
    col = np.ascontiguousarray(col)
    pos = np.zeros(max(len(col), 1), dtype=np.uint64)
    c = C.c_uint64()
    _check("leco_ref_start_positions_delta", lib().leco_ref_start_positions_delta(
        _ptr(col), len(col), _dtype_code(col), _ptr(pos), C.byref(c)))
    return pos[: c.value].copy()


def partition_merge(col: np.ndarray, starts, max_len: int = 1 << 20,
                    max_passes: int = 0) -> np.ndarray:
    """Merge scan (section 3.2.2) applied to the partitioning `starts`."""
    col = np.ascontiguousarray(col)
    s = np.array(starts, dtype=np.uint64)
    m = C.c_uint64(len(s) - 1)
    _check("leco_ref_partition_merge", lib().leco_ref_partition_merge(
        _ptr(col), len(col), _dtype_code(col), _ptr(s), C.byref(m), max_len, max_passes))
    return s[: m.value + 1].copy()


def delta_fix_bytes(col: np.ndarray, L: int) -> int:
    """Size of the Delta-fix encoding (section 2, Delta over fixed partitions)."""
    col = np.ascontiguousarray(col)
    b = C.c_uint64()
    _check("leco_ref_delta_fix_bytes", lib().leco_ref_delta_fix_bytes(
        _ptr(col), len(col), _dtype_code(col), L, C.byref(b)))
    return b.value


def delta_fix_encode(col: np.ndarray, L: int) -> np.ndarray:
    col = np.ascontiguousarray(col)
    size = delta_fix_bytes(col, L)
    out = np.zeros(max(size, 1), dtype=np.uint8)
    b = C.c_uint64()
    _check("leco_ref_delta_fix_encode", lib().leco_ref_delta_fix_encode(
        _ptr(col), len(col), _dtype_code(col), L, _ptr(out), size, C.byref(b)))
    return out[: b.value].copy()


def delta_fix_decode(blob: np.ndarray) -> np.ndarray:
    blob = np.ascontiguousarray(blob, dtype=np.uint8)
    n = int(blob[8:16].view(np.uint64)[0])
    out = np.zeros(max(n, 1), dtype=_np_dtype(int(blob[6])))
    _check("leco_ref_delta_fix_decode", lib().leco_ref_delta_fix_decode(
        _ptr(blob), len(blob), _ptr(out), n))
    return out[:n].copy()


def partition_dp(col: np.ndarray, max_len: int = 1 << 20) -> tuple[np.ndarray, int]:
    col = np.ascontiguousarray(col)
    starts = np.zeros(len(col) + 1, dtype=np.uint64)
    m, b = C.c_uint64(), C.c_uint64()
    _check("leco_ref_partition_dp", lib().leco_ref_partition_dp(
        _ptr(col), len(col), _dtype_code(col), max_len, _ptr(starts), C.byref(m),
        C.byref(b)))
    return starts[: m.value + 1].copy(), b.value


def partition_bruteforce(col: np.ndarray, max_len: int = 1 << 20) -> tuple[np.ndarray, int]:
    col = np.ascontiguousarray(col)
    starts = np.zeros(len(col) + 1, dtype=np.uint64)
    m, b = C.c_uint64(), C.c_uint64()
    _check("leco_ref_partition_bruteforce", lib().leco_ref_partition_bruteforce(
        _ptr(col), len(col), _dtype_code(col), max_len, _ptr(starts), C.byref(m),
        C.byref(b)))
    return starts[: m.value + 1].copy(), b.value


def partitioning_cost(col: np.ndarray, starts) -> int:
    col = np.ascontiguousarray(col)
    s = np.ascontiguousarray(starts, dtype=np.uint64)
    b = C.c_uint64()
    _check("leco_ref_partitioning_cost", lib().leco_ref_partitioning_cost(
        _ptr(col), len(col), _dtype_code(col), _ptr(s), len(s) - 1, C.byref(b)))
    return b.value


def fixed_cost(col: np.ndarray, starts, window: int, L: int, regressor: str = "ls") -> int:
    """Sampled cost of fixed partitions of length L (record + word bytes of
    every partition of every window)."""
    col = np.ascontiguousarray(col)
    s = np.ascontiguousarray(starts, dtype=np.uint64)
    out = C.c_uint64()
    _check("leco_ref_fixed_cost", lib().leco_ref_fixed_cost(
        _ptr(col), len(col), _dtype_code(col), _ptr(s), len(s), window, L,
        _regressor(regressor), C.byref(out)))
    return out.value


def _search_result(L, cost, trace, tl) -> dict:
    steps = [(int(trace[2 * i]), int(trace[2 * i + 1])) for i in range(min(tl.value, len(trace) // 2))]
    return {"L": L.value, "cost": cost.value, "trace": steps}


def size_search_fn(window: int, cost) -> dict:
    """The size search over a Python cost function L -> int."""
    cb = COST_FN(lambda _ctx, L: int(cost(int(L))))
    L, c, tl = C.c_uint64(), C.c_uint64(), C.c_uint64()
    trace = np.zeros(2 * 4096, dtype=np.uint64)
    _check("leco_ref_size_search_fn", lib().leco_ref_size_search_fn(
        window, cb, None, C.byref(L), C.byref(c), _ptr(trace), len(trace), C.byref(tl)))
    return _search_result(L, c, trace, tl)


def size_search(col: np.ndarray, starts, window: int, regressor: str = "ls") -> dict:
    """Fixed partition size search (section 3.2.1) over sampled windows."""
    col = np.ascontiguousarray(col)
    s = np.ascontiguousarray(starts, dtype=np.uint64)
    L, c, tl = C.c_uint64(), C.c_uint64(), C.c_uint64()
    trace = np.zeros(2 * 4096, dtype=np.uint64)
    _check("leco_ref_size_search", lib().leco_ref_size_search(
        _ptr(col), len(col), _dtype_code(col), _ptr(s), len(s), window, _regressor(regressor),
        C.byref(L), C.byref(c), _ptr(trace), len(trace), C.byref(tl)))
    return _search_result(L, c, trace, tl)
