"""Seeded synthetic inputs shaped like the LeCo paper's integer workloads.

This module only draws inputs; it holds none of the codec's arithmetic and is
shared by the tests, the benchmark and the smoke check, which hand the same
arrays to the GPU path and to the CPU oracle.

The paper's data sets (sorted 200M-key SOSD-style sets, piecewise-linear ID
columns, columns with runs of repeated values; section 4.1) are not
available, so each generator reproduces the described shape instead:

* ``linear_noise``  v_i = 1000 + 7 i + U{0..63}                   (fixed L=1024)
* ``lognormal_keys`` sorted keys, cumulative sum of max(1, rint(lognormal(3, 1.5)))
* ``sorted_normal`` sorted samples of N(2^30, 2^26) clipped to uint32
* ``piecewise_linear`` 1000 random segments, slopes U[0, 50), noise U{0..255}
* ``constant_runs`` runs of one value, geometric run lengths with mean 64
"""
from __future__ import annotations

import numpy as np

U32_MAX = (1 << 32) - 1

# Workload sizes and seeds.
C1_N, C1_L, C1_SEED, C1_RA, C1_RA_SEED = 1_000_000, 1024, 1, 100_000, 11
C2_N, C2_L, C2_SEED, C2_RA, C2_RA_SEED = 200_000_000, 4096, 2, 100_000_000, 21
C3_N, C3_SEEDS = 100_000_000, (31, 32, 33)
C4_COLS, C4_SEED = 4096, 41
C5_COLS, C5_N, C5_SEED = 64, 39_062_500, 51


def linear_noise(n: int = C1_N, seed: int = C1_SEED, dtype=np.uint64) -> np.ndarray:
    """v_i = 1000 + 7*i + U{0..63}."""
    rng = np.random.default_rng(seed)
    i = np.arange(n, dtype=np.uint64)
    v = np.uint64(1000) + np.uint64(7) * i + rng.integers(0, 64, size=n, dtype=np.uint64)
    return v.astype(dtype)


def lognormal_keys(n: int = C2_N, seed: int = C2_SEED, dtype=np.uint64) -> np.ndarray:
    """Sorted keys: cumulative sum of integer gaps max(1, rint(lognormal(3, 1.5)))."""
    rng = np.random.default_rng(seed)
    g = np.rint(rng.lognormal(3.0, 1.5, size=n))
    np.maximum(g, 1.0, out=g)
    keys = np.cumsum(g.astype(np.uint64))
    if dtype == np.uint32:
        assert n == 0 or int(keys[-1]) <= U32_MAX, "keys overflow uint32"
    return keys.astype(dtype, copy=False)


def sorted_normal(n: int = C3_N, seed: int = C3_SEEDS[0]) -> np.ndarray:
    """Sorted samples of N(2^30, std 2^26), rounded and clipped to uint32."""
    rng = np.random.default_rng(seed)
    x = np.rint(rng.normal(float(1 << 30), float(1 << 26), size=n))
    np.clip(x, 0, U32_MAX, out=x)
    x.sort()
    return x.astype(np.uint32)


def piecewise_linear(n: int = C3_N, seed: int = C3_SEEDS[1], segments: int = 1000) -> np.ndarray:
    """Continuous polyline from 0 over `segments` random pieces with slopes in
    U[0, 50), plus integer noise U{0..255}."""
    rng = np.random.default_rng(seed)
    cuts = np.sort(rng.choice(np.arange(1, n), size=min(segments - 1, max(n - 1, 0)),
                              replace=False)) if n > 1 else np.zeros(0, dtype=np.int64)
    bounds = np.concatenate([[0], cuts, [n]]).astype(np.int64)
    slopes = rng.uniform(0.0, 50.0, size=len(bounds) - 1)
    y = np.empty(n, dtype=np.float64)
    level = 0.0
    for s, a, b in zip(slopes, bounds[:-1], bounds[1:]):
        y[a:b] = level + s * np.arange(b - a, dtype=np.float64)
        level += s * (b - a)
    v = np.floor(y).astype(np.uint64) + rng.integers(0, 256, size=n, dtype=np.uint64)
    assert n == 0 or int(v.max()) <= U32_MAX, "piecewise column overflows uint32"
    return v.astype(np.uint32)


def constant_runs(n: int = C3_N, seed: int = C3_SEEDS[2], mean_run: int = 64) -> np.ndarray:
    """Runs of one uniform uint32 value with Geometric(1/mean_run) lengths."""
    rng = np.random.default_rng(seed)
    out = np.empty(n, dtype=np.uint32)
    filled = 0
    while filled < n:
        k = max(16, (n - filled) // mean_run + 16)
        runs = rng.geometric(1.0 / mean_run, size=k)
        vals = rng.integers(0, 1 << 32, size=k, dtype=np.uint64).astype(np.uint32)
        chunk = np.repeat(vals, runs)[: n - filled]
        out[filled: filled + len(chunk)] = chunk
        filled += len(chunk)
    return out


def uniform_positions(n: int, k: int, seed: int) -> np.ndarray:
    """k uniform random positions in [0, n)."""
    rng = np.random.default_rng(seed)
    return rng.integers(0, n, size=k, dtype=np.uint64)


def batched_columns(ncols: int = C4_COLS, seed: int = C4_SEED, lo: float = 1e3,
                    hi: float = 1e7, median: float = 1.3e5, sigma: float = 1.7):
    """Column specs for the batched workload: lognormal lengths clipped to
    [lo, hi]; per column uint32 or uint64 and a linear-noise (L=1024) or
    lognormal-keys (L=4096) generator, each with its own seed.  Returns a
    list of dicts; call ``make_column`` to draw one."""
    rng = np.random.default_rng(seed)
    lens = np.clip(np.rint(np.exp(rng.normal(np.log(median), sigma, size=ncols))), lo, hi)
    specs = []
    for c in range(ncols):
        specs.append(dict(
            n=int(lens[c]),
            dtype=np.uint32 if rng.integers(0, 2) == 0 else np.uint64,
            kind="linear_noise" if rng.integers(0, 2) == 0 else "lognormal_keys",
            seed=int(rng.integers(0, 2**31)),
        ))
    for s in specs:
        s["fixed_len"] = C1_L if s["kind"] == "linear_noise" else C2_L
    return specs


def make_column(spec: dict) -> np.ndarray:
    if spec["kind"] == "linear_noise":
        return linear_noise(spec["n"], spec["seed"], spec["dtype"])
    return lognormal_keys(spec["n"], spec["seed"], spec["dtype"])


def filter_bounds(col: np.ndarray) -> tuple[int, int]:
    """[vmin + R/4, vmin + 3R/4) for a column with range R = vmax - vmin."""
    vmin, vmax = int(col.min()), int(col.max())
    r = vmax - vmin
    return vmin + r // 4, vmin + (3 * r) // 4


def served_columns(ncols: int = C5_COLS, n: int = C5_N, seed: int = C5_SEED):
    """Column specs for the served workload: uint64 columns alternating the
    linear-noise and lognormal-keys generators."""
    rng = np.random.default_rng(seed)
    specs = []
    for c in range(ncols):
        kind = "linear_noise" if c % 2 == 0 else "lognormal_keys"
        specs.append(dict(n=n, dtype=np.uint64, kind=kind, seed=int(rng.integers(0, 2**31)),
                          fixed_len=C1_L if kind == "linear_noise" else C2_L))
    return specs


def request_stream(num: int, col_lens, seed: int = C5_SEED + 1, rate: float = 1.0):
    """Poisson request stream: arrival times (seconds, mean gap 1/rate), half
    random-access batches of floor(2^U[0,16]) positions, half range scans of
    floor(10^U[3,7]) values, each on a uniform column."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=num)
    t = np.cumsum(gaps)
    reqs = []
    for q in range(num):
        c = int(rng.integers(0, len(col_lens)))
        n = int(col_lens[c])
        if rng.integers(0, 2) == 0:
            k = int(np.floor(2.0 ** rng.uniform(0, 16)))
            pos = rng.integers(0, n, size=k, dtype=np.uint64)
            reqs.append(dict(t=float(t[q]), kind="ra", col=c, positions=pos))
        else:
            ln = min(int(np.floor(10.0 ** rng.uniform(3, 7))), n)
            b = int(rng.integers(0, n - ln + 1))
            reqs.append(dict(t=float(t[q]), kind="range", col=c, begin=b, end=b + ln))
    return reqs


# ---- device-side generators for the multi-gigabyte workloads ---------------------
# Drawing 2e9 values on the host takes minutes, so the batched and served
# workloads draw each column on the GPU with torch's seeded Philox generator
# (one seed per column).  Same shapes as the host generators above; 32-bit
# columns are returned as int32 tensors holding the uint32 bit patterns
# (every generated value is below 2^31), 64-bit columns as int64.

def _torch_gen(seed: int, device):
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    return g


def linear_noise_device(n: int, seed: int, dtype, device="cuda"):
    import torch
    g = _torch_gen(seed, device)
    v = torch.arange(n, dtype=torch.int64, device=device) * 7 + 1000
    v += torch.randint(0, 64, (n,), generator=g, device=device, dtype=torch.int64)
    return v.to(torch.int32) if dtype == np.uint32 else v


def lognormal_keys_device(n: int, seed: int, dtype, device="cuda"):
    import torch
    g = _torch_gen(seed, device)
    x = torch.randn(n, generator=g, device=device, dtype=torch.float64)
    gaps = torch.round(torch.exp(x * 1.5 + 3.0)).clamp_(min=1.0).to(torch.int64)
    keys = torch.cumsum(gaps, 0)
    if dtype == np.uint32:
        assert n == 0 or int(keys[-1]) < 2**31, "keys overflow the 32-bit column"
        return keys.to(torch.int32)
    return keys


def make_column_device(spec: dict, device="cuda"):
    if spec["kind"] == "linear_noise":
        return linear_noise_device(spec["n"], spec["seed"], spec["dtype"], device)
    return lognormal_keys_device(spec["n"], spec["seed"], spec["dtype"], device)


def request_mix(num: int, col_lens, seed: int, max_log2_k: float = 16.0,
                range_exp=(3.0, 7.0), rate: float = 1.0):
    """Same shape as ``request_stream`` with adjustable size limits:
    random-access batches of floor(2^U[0, max_log2_k]) positions and range
    scans of floor(10^U[range_exp]) values."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, size=num))
    reqs = []
    for q in range(num):
        c = int(rng.integers(0, len(col_lens)))
        n = int(col_lens[c])
        if rng.integers(0, 2) == 0:
            k = int(np.floor(2.0 ** rng.uniform(0, max_log2_k)))
            reqs.append(dict(t=float(t[q]), kind="ra", col=c,
                             positions=rng.integers(0, n, size=k, dtype=np.uint64)))
        else:
            ln = min(int(np.floor(10.0 ** rng.uniform(*range_exp))), n)
            b = int(rng.integers(0, n - ln + 1))
            reqs.append(dict(t=float(t[q]), kind="range", col=c, begin=b, end=b + ln))
    return reqs


def sample_window_starts(n: int, window: int, fraction: float = 0.01, seed: int = 61) -> np.ndarray:
    """Starts of the sampled windows of the fixed partition size search: k =
    max(1, floor(fraction * n / window)) uniform starts in [0, n - window]
    (sorted), so about `fraction` of the column is sampled."""
    k = max(1, int(fraction * n) // window)
    rng = np.random.default_rng(seed)
    return np.sort(rng.integers(0, n - window + 1, size=k)).astype(np.uint64)


def cosmos(n: int, seed: int = 71) -> np.ndarray:
    """Higher-order signal of the evaluation's non-linear data (a cosmic-ray
    like mixture of two sines plus Gaussian noise):
    (sin((x + 10) / (60 pi)) + sin(3 (x + 10) / (60 pi)) / 10) * 10^6 +
    N(0, 100) (read as standard deviation 100), shifted by 2^21 so every
    value is a non-negative uint32."""
    rng = np.random.default_rng(seed)
    x = np.arange(n, dtype=np.float64) + 10.0
    w = 60.0 * np.pi
    y = (np.sin(x / w) + np.sin(3.0 * x / w) / 10.0) * 1e6 + rng.normal(0.0, 100.0, n)
    return np.rint(y + float(1 << 21)).astype(np.uint32)


def poly_blocks(n: int, seed: int = 72, lo: int = 1000, hi: int = 8000) -> np.ndarray:
    """Blocks of U[lo, hi) values, each following its own cubic polynomial
    a + b t + c t^2 + d t^3 of the block-local index (b in [0, 1000), c in
    [-0.05, 0.05), d in [-1e-5, 1e-5), a continuing from the previous block)
    plus U{0..15} noise; 64-bit values offset by 2^40."""
    rng = np.random.default_rng(seed)
    out = np.empty(n, dtype=np.uint64)
    i, a = 0, float(1 << 40)
    while i < n:
        ln = min(n - i, int(rng.integers(lo, hi)))
        t = np.arange(ln, dtype=np.float64)
        b, c, d = rng.uniform(0, 1000), rng.uniform(-0.05, 0.05), rng.uniform(-1e-5, 1e-5)
        y = a + b * t + c * t * t + d * t * t * t
        out[i:i + ln] = np.rint(y).astype(np.uint64) + rng.integers(0, 16, ln).astype(np.uint64)
        a = float(y[-1])
        i += ln
    return out
