"""From-scratch Python restatements of the variable-length partitioner
(section 3.2.2), used to pin the C oracle's split, starting partitions and
merge scan on small columns.  Everything here is recomputed from the
definitions, non-incrementally, with Python integers: no state carried
between inclusion decisions, no code shared with the oracle.

The size of a partition (what the merge compares) is the exact number of
bytes it costs in a variable-length blob: a 32-byte record, an 8-byte start
and its residual words, ceil(len * b / 64) * 8 bytes, where b is the width
the encoder stores: the least-squares line (section 3.1) with its slope
fl(N) / fl(D) from exact integer sums, predictions floor(theta1 * t), and
the constant model (FOR, section 2) whenever that is not wider.
"""
from __future__ import annotations

import math


def delta_tilde(v, i: int, j: int) -> int:
    """D~(v[i, j)) for the linear regressor: bitlen(max d - min d) over the
    first differences d_k = v_k - v_{k-1}, k = i+1 .. j-1 (0 without two
    values)."""
    ds = [int(v[k]) - int(v[k - 1]) for k in range(i + 1, j)]
    return (max(ds) - min(ds)).bit_length() if ds else 0


def inclusion_cost(v, i: int, j: int) -> int:
    """C = (j + 1 - i) D~(v[i, j+1)) - (j - i) D~(v[i, j)): the cost of
    appending v[j] to the partition v[i, j)."""
    return (j + 1 - i) * delta_tilde(v, i, j + 1) - (j - i) * delta_tilde(v, i, j)


def starting_partitions(v) -> list[tuple[int, int]]:
    """Segments of smallest second-order delta |v_k - 2 v_{k-1} + v_{k-2}|
    (degree 1 + 1): each maximal run k..k' of positions at the column's
    minimum gives the starting partition [k - 2, k' + 1); of two that would
    share a value, the later keeps it."""
    n = len(v)
    if n < 3:
        return []
    dd = {k: abs(int(v[k]) - 2 * int(v[k - 1]) + int(v[k - 2])) for k in range(2, n)}
    best = min(dd.values())
    good = [k for k in range(2, n) if dd[k] == best]
    runs, k = [], 0
    while k < len(good):
        e = k
        while e + 1 < len(good) and good[e + 1] == good[e] + 1:
            e += 1
        runs.append([good[k] - 2, good[e] + 1])
        k = e + 1
    for a, b in zip(runs, runs[1:]):
        if b[0] < a[1]:
            a[1] = b[0]
    return [(a, b) for a, b in runs]


def split(v, tau: float, sm_bits: int, max_len: int = 1 << 20, starting=None) -> list[int]:
    """The split phase: left to right, v[j] joins the current partition v[i, j)
    while len = j - i < max_len and C <= tau * S_M; with starting partitions,
    each one's first value begins a partition and its other values join
    without the cost test."""
    n = len(v)
    if n == 0:
        return [0]
    first, inside = set(), set()
    for a, b in starting or []:
        first.add(a)
        inside.update(range(a + 1, b))
    starts, i = [0], 0
    for j in range(1, n):
        length = j - i
        if length < max_len and j not in first and (
                j in inside or inclusion_cost(v, i, j) <= tau * sm_bits):
            continue
        starts.append(j)
        i = j
    return starts + [n]


def encoder_bits(y) -> int:
    """Residual width the encoder stores for one partition y (Python ints)."""
    n = len(y)
    vmin, vmax = min(y), max(y)
    b_for = (vmax - vmin).bit_length()
    if n == 1 or vmax - vmin >= 1 << 61:
        return b_for
    yy = [x - vmin for x in y]
    s_t, s_tt = n * (n - 1) // 2, (n - 1) * n * (2 * n - 1) // 6
    s_y, s_ty = sum(yy), sum(t * x for t, x in enumerate(yy))
    num, den = n * s_ty - s_t * s_y, n * s_tt - s_t * s_t
    theta = float(num) / float(den)  # each int rounded to nearest, one division
    if theta == 0.0:
        theta = 0.0
    r = [x - math.floor(theta * float(t)) for t, x in enumerate(yy)]
    b_ls = (max(r) - min(r)).bit_length()
    return b_for if b_for <= b_ls else b_ls


def size_bytes(v, a: int, b: int) -> int:
    """Bytes v[a, b) costs in a variable-length blob."""
    bits = encoder_bits([int(x) for x in v[a:b]])
    return 32 + 8 + 8 * (((b - a) * bits + 63) // 64)


def merge(v, starts, max_len: int = 1 << 20, max_passes: int = 0) -> list[int]:
    """The merge phase: scan the partitions from the left; the current one
    merges with its right neighbour when the union is strictly smaller and
    fits max_len, and then tries the next neighbour; passes repeat until one
    merges nothing (or max_passes passes)."""
    s = [int(x) for x in starts]
    passes = 0
    while len(s) > 2 and (max_passes == 0 or passes < max_passes):
        merged = False
        out = [s[0]]
        for k in range(1, len(s) - 1):
            a, b, c = out[-1], s[k], s[k + 1]
            if c - a <= max_len and size_bytes(v, a, c) < size_bytes(v, a, b) + size_bytes(v, b, c):
                merged = True
                continue
            out.append(b)
        out.append(s[-1])
        s = out
        passes += 1
        if not merged:
            break
    return s
