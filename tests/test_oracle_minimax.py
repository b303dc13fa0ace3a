"""Pins of the oracle's minimax regressor (section 3.1's fixed-width
objective) against brute force over exact fractions, closed forms and
invariances.  CPU only."""
from __future__ import annotations

from fractions import Fraction

import numpy as np
import pytest


def strip_width(v, theta: Fraction) -> Fraction:
    """Vertical width of the thinnest strip of slope theta holding every
    point (t, v_t)."""
    d = [Fraction(int(x)) - theta * t for t, x in enumerate(v)]
    return max(d) - min(d)


def brute_force_slope(v) -> Fraction:
    """The smallest slope minimising the strip width, searched over every
    slope through two of the points.  The width is convex and piecewise
    linear in the slope and bends only at such slopes, so the left end of
    its set of minimisers is one of them."""
    n = len(v)
    cands = sorted({Fraction(int(v[j]) - int(v[i]), j - i) for i in range(n) for j in range(i + 1, n)})
    widths = [strip_width(v, c) for c in cands]
    best = min(widths)
    return next(c for c, w in zip(cands, widths) if w == best)


def tiny_columns(rng):
    for n in range(2, 11):
        for _ in range(25):
            kind = rng.integers(0, 5)
            if kind == 0:
                v = rng.integers(0, 20, n)
            elif kind == 1:  # near a line, either direction
                v = 1000 + rng.integers(-9, 10) * np.arange(n) + rng.integers(0, 4, n)
            elif kind == 2:  # many ties and collinear triples
                v = 3 * np.arange(n) + 5 * (rng.integers(0, 2, n))
            elif kind == 3:  # large values, differences near 2^60
                v = (1 << 62) + rng.integers(0, 1 << 60, n, dtype=np.int64)
            else:
                v = np.full(n, rng.integers(0, 100))
            yield np.asarray(v, dtype=np.uint64)


def test_minimax_slope_equals_brute_force(ref):
    rng = np.random.default_rng(71)
    count = 0
    for v in tiny_columns(rng):
        dy, dt = ref.minimax_slope(v)
        assert dt > 0
        assert Fraction(dy, dt) == brute_force_slope(v), v.tolist()
        count += 1
    assert count == 9 * 25


def test_no_other_slope_is_narrower(ref):
    """Probes slopes between and beyond the candidates: none gives a
    thinner strip than the returned slope, and none below it gives an equal
    one."""
    rng = np.random.default_rng(72)
    for _ in range(60):
        n = int(rng.integers(2, 12))
        v = np.asarray(rng.integers(0, 50, n), dtype=np.uint64)
        dy, dt = ref.minimax_slope(v)
        th = Fraction(dy, dt)
        w = strip_width(v, th)
        for k in range(-40, 41):
            probe = th + Fraction(k, 7)
            pw = strip_width(v, probe)
            assert pw >= w
            if probe < th:
                assert pw > w


def test_two_points_give_their_slope(ref):
    assert ref.minimax_slope(np.array([5, 17], dtype=np.uint64)) == (12, 1)
    dy, dt = ref.minimax_slope(np.array([17, 5], dtype=np.uint64))
    assert Fraction(dy, dt) == -12


def test_line_with_one_spike_keeps_the_line(ref):
    """Points of v = 10 t + 10 with one point raised by h: for any other
    slope the spike or an end point moves farther out, so the minimax slope
    is 10 and the width is h (exactly bitlen(h) bits), while least squares
    tilts towards the spike: its residual range exceeds h, and with h just
    under 2^10 that costs an eleventh bit."""
    n, h, k = 64, 1020, 5
    v = 10 * np.arange(n, dtype=np.uint64) + np.uint64(10)
    v[k] += np.uint64(h)
    dy, dt = ref.minimax_slope(v)
    assert Fraction(dy, dt) == 10
    md = ref.fit(v, regressor="minimax")
    assert md["theta1_mm"] == 10.0
    assert md["r_max_mm"] - md["r_min_mm"] == h
    assert md["b_mm"] == h.bit_length()
    assert md["theta1_ls"] != 10.0
    assert md["r_max"] - md["r_min"] > h
    assert md["b_ls"] == 11 and md["b_mm"] == 10
    assert md["mode"] == 2 and md["bits"] == md["b_mm"] and md["theta1"] == 10.0


@pytest.mark.parametrize("n", [5, 8, 33, 64])
def test_convex_sequence_takes_the_chord(ref, n):
    """v_t = t^2: the upper hull is the single chord from t = 0 to n - 1,
    every point is a lower-hull vertex, and the thinnest strip is parallel
    to the chord (slope n - 1).  When n - 1 is odd a lower edge t -> t + 1
    has the same slope 2t + 1 = n - 1; the bend is reported as the upper
    edge's fraction ((n-1)^2, n-1)."""
    v = np.arange(n, dtype=np.uint64) ** 2
    assert ref.minimax_slope(v) == ((n - 1) ** 2, n - 1)


def test_adding_a_line_shifts_the_slope(ref):
    """W_{v + c t + a}(theta) = W_v(theta - c), so the smallest minimiser
    moves by exactly c; a constant shift changes nothing."""
    rng = np.random.default_rng(73)
    for _ in range(40):
        n = int(rng.integers(2, 300))
        v = np.asarray(rng.integers(0, 1 << 20, n), dtype=np.uint64) + np.uint64(1 << 40)
        dy, dt = ref.minimax_slope(v)
        c = int(rng.integers(-1000, 1000))
        a = int(rng.integers(0, 1 << 30))
        w = np.array([int(x) + c * t + a for t, x in enumerate(v)], dtype=np.uint64)
        dy2, dt2 = ref.minimax_slope(w)
        assert Fraction(dy2, dt2) == Fraction(dy, dt) + c


def test_model_choice_and_tie_order(ref):
    """With the minimax regressor the stored width is min(b_for, b_ls,
    b_mm); the minimax line is stored only when strictly narrower than both
    others, and its residuals are those of floor(theta1_mm * t)."""
    rng = np.random.default_rng(74)
    seen = set()
    for _ in range(300):
        n = int(rng.integers(1, 200))
        kind = rng.integers(0, 3)
        if kind == 0:
            v = rng.integers(0, 1 << 12, n)
        elif kind == 1:
            v = 5 * np.arange(n) + rng.integers(0, 64, n)
            v[rng.integers(0, n)] += int(rng.integers(0, 5000))
        else:
            v = np.cumsum(rng.integers(1, 100, n))
        v = np.asarray(v, dtype=np.uint64)
        ls = ref.fit(v)
        mm = ref.fit(v, regressor="minimax")
        for key in ("vmin", "b_for", "theta1_ls", "b_ls"):
            assert ls[key] == mm[key]
        if n == 1:
            assert mm["mm_fitted"] == 0 and mm["mode"] == 0
            continue
        assert mm["mm_fitted"] == 1
        th = mm["theta1_mm"]
        r = [int(x) - mm["vmin"] - int(np.floor(th * t)) for t, x in enumerate(v)]
        assert (min(r), max(r)) == (mm["r_min_mm"], mm["r_max_mm"])
        assert mm["b_mm"] == (max(r) - min(r)).bit_length()
        assert mm["bits"] == min(mm["b_for"], mm["b_ls"], mm["b_mm"])
        want = 2 if mm["b_mm"] < min(mm["b_for"], mm["b_ls"]) else ls["mode"]
        assert mm["mode"] == want
        seen.add(want)
    assert seen == {0, 1, 2}


def test_minimax_blobs_round_trip_and_never_grow(ref):
    from paper_2306_15374_amd import workloads as W
    cols = [W.linear_noise(20_000, 1), W.lognormal_keys(20_000, 2),
            W.piecewise_linear(20_000, 3, segments=20).astype(np.uint32), W.constant_runs(20_000, 4)]
    for col in cols:
        for L in (64, 1000):
            ls = ref.encode(col, fixed_len=L)
            mm = ref.encode(col, fixed_len=L, regressor="minimax")
            assert np.array_equal(ref.decode_all(mm), col)
            assert len(mm) <= len(ls)
            assert ref.blob_bytes(col, fixed_len=L, regressor="minimax") == len(mm)


def test_minimax_rejects_bad_arguments(ref):
    import oracle
    with pytest.raises(oracle.OracleError):
        ref.minimax_slope(np.array([3], dtype=np.uint64))
    with pytest.raises(oracle.OracleError):
        ref.minimax_slope(np.array([0, 1 << 61], dtype=np.uint64))
    with pytest.raises(ValueError):
        ref.fit(np.arange(4, dtype=np.uint64), regressor="cubic")
