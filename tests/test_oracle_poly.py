"""Pins of the oracle's polynomial regressor (degree 2 and 3 least squares
in the discrete orthogonal basis): leading coefficients against exact
normal-equation solves in the monomial basis, exact polynomial data, the
model choice, the blob layout and round trips.  CPU only."""
from __future__ import annotations

from fractions import Fraction

import numpy as np
import pytest

from paper_2306_15374_amd import workloads as W


def exact_lstsq(y, degree: int):
    """Least-squares polynomial coefficients (monomial basis, lowest first)
    by Gauss-Jordan elimination over exact fractions."""
    n = len(y)
    A = [[Fraction(sum(t ** (i + j) for t in range(n))) for j in range(degree + 1)]
         for i in range(degree + 1)]
    b = [Fraction(sum(int(y[t]) * t ** i for t in range(n))) for i in range(degree + 1)]
    m = len(A)
    for c in range(m):
        p = next(r for r in range(c, m) if A[r][c] != 0)
        A[c], A[p], b[c], b[p] = A[p], A[c], b[p], b[c]
        for r in range(m):
            if r != c and A[r][c] != 0:
                f = A[r][c] / A[c][c]
                A[r] = [x - f * z for x, z in zip(A[r], A[c])]
                b[r] -= f * b[c]
    return [b[i] / A[i][i] for i in range(m)]


def close(x: float, q: Fraction, ulps: int = 4) -> bool:
    """|x - q| within a few units in the last place of x (three roundings)."""
    if q == 0:
        return x == 0
    return abs(Fraction(x) - q) <= ulps * Fraction(np.spacing(abs(float(q))))


@pytest.mark.parametrize("seed", range(5))
def test_leading_coefficients_are_exact_least_squares(ref, seed):
    """The Gram polynomials have leading coefficients 2, 6 and 20 and lower
    degrees below them, so the least-squares polynomial of degree k has
    monomial leading coefficient 2 c1 (k = 1), 6 c2 (k = 2), 20 c3 (k = 3)
    in terms of the oracle's coefficients."""
    rng = np.random.default_rng(seed)
    for n in (4, 5, 9, 17, 40):
        y = rng.integers(0, 1 << 20, n)
        if seed % 2:
            t = np.arange(n)
            y = 1000 + 3 * t * t - 2 * t + rng.integers(0, 50, n)
        v = np.asarray(y, dtype=np.uint64)
        md = ref.fit(v, regressor="poly")
        assert md["poly_fitted"] == 1
        c1, c2, c3 = md["pc"]
        assert close(2 * c1, exact_lstsq(v, 1)[1])
        assert close(6 * c2, exact_lstsq(v, 2)[2])
        assert close(20 * c3, exact_lstsq(v, 3)[3])


def test_degree_one_coefficient_matches_the_fitted_line(ref):
    rng = np.random.default_rng(7)
    for n in (3, 10, 1000, 4096):
        v = np.asarray(rng.integers(0, 1 << 30, n), dtype=np.uint64)
        md = ref.fit(v, regressor="poly")
        # 2 c1 and fl(N)/fl(D) are the same rational rounded along two paths
        assert abs(2 * md["pc"][0] - md["theta1_ls"]) <= 4 * np.spacing(abs(md["theta1_ls"]))


@pytest.mark.parametrize("coef", [(1000, 7, 0, 0), (5, -3, 2, 0), (1 << 40, 11, -5, 1), (0, 0, 0, 2)])
def test_exact_polynomials_fit_within_a_bit(ref, coef):
    """Integer polynomial data of degree <= 3 on 4096 points: the fit is the
    data itself up to rounding, so the residual range is at most 1 (floor of
    a value within a few ulps of an integer)."""
    a, b, c, d = coef
    t = np.arange(4096, dtype=object)
    v = np.array([a + b * x + c * x * x + d * x ** 3 + (1 << 36) for x in t], dtype=np.uint64)
    md = ref.fit(v, regressor="poly")
    assert md["b_p3"] <= 1
    assert md["bits"] <= 1


def test_model_choice_and_tie_order(ref):
    """The stored width is min(b_for, b_ls, b_p2, b_p3); a polynomial is
    stored only when strictly narrower than every simpler model, degree 3
    only when strictly narrower than degree 2; the residual range of the
    stored polynomial is recomputed here from its coefficients."""
    rng = np.random.default_rng(8)
    seen = set()
    for _ in range(300):
        n = int(rng.integers(1, 400))
        kind = rng.integers(0, 4)
        t = np.arange(n)
        if kind == 0:
            v = rng.integers(0, 1 << 10, n)
        elif kind == 1:
            v = 9 * t + rng.integers(0, 30, n)
        elif kind == 2:
            v = (t * t) // 3 + rng.integers(0, 4, n)
        else:
            v = (t ** 3) // 50 - 7 * t * t + 2_000_000 + rng.integers(0, 4, n)
        v = np.asarray(v, dtype=np.uint64)
        md = ref.fit(v, regressor="poly")
        ls = ref.fit(v)
        assert md["b_ls"] == ls["b_ls"] and md["b_for"] == ls["b_for"]
        if n < 3:
            assert md["poly_fitted"] == 0 and md["mode"] == ls["mode"]
            continue
        b2, b3 = md["b_p2"], md["b_p3"]
        if n < 4:
            assert b3 == 99
        assert md["bits"] == min(md["b_for"], md["b_ls"], b2, b3)
        if md["mode"] == 3:
            assert min(b2, b3) < min(md["b_for"], md["b_ls"])
            deg = 3 if b3 < b2 else 2
            assert md["poly_degree"] == deg
            c = md["stored_c"]
            assert (c[2] == 0.0) == (deg == 2)
        else:
            assert md["mode"] == ls["mode"]
        seen.add(md["mode"] * 10 + md["poly_degree"])
    assert {0, 10, 32, 33} <= seen


def test_eligibility_limits(ref):
    """No polynomial for fewer than 3 values, more than 4096, or a range of
    2^50 or more; degree 3 needs 4 values."""
    t = np.arange(5000, dtype=np.uint64)
    sq = t * t
    assert ref.fit(sq[:4096], regressor="poly")["poly_fitted"] == 1
    assert ref.fit(sq[:4097], regressor="poly")["poly_fitted"] == 0
    assert ref.fit(sq[:2], regressor="poly")["poly_fitted"] == 0
    assert ref.fit(sq[:3], regressor="poly")["b_p3"] == 99
    wide = np.array([0, 1 << 50, 5, 9], dtype=np.uint64)
    assert ref.fit(wide, regressor="poly")["poly_fitted"] == 0
    assert ref.fit(wide - np.uint64(1) + np.array([1, 0, 0, 0], dtype=np.uint64),
                   regressor="poly")["poly_fitted"] == 1


def parse(blob):
    h = blob[:64].view(np.uint64)
    return {"flags": int(blob[7]), "m": int(h[2]), "starts_off": int(h[5]),
            "words_off": int(h[6]), "total_words": int(h[7])}


@pytest.mark.parametrize("variable", [False, True])
def test_blob_layout_with_coefficients(ref, variable):
    """Flag bit 1, the (c2, c3) section right after the records (and
    starts) at a 16-byte boundary, words after it; kind bytes 0/1 with zero
    coefficients for kind 0; c1 in the slope field."""
    rng = np.random.default_rng(9)
    col = W.cosmos(30_000, 10)
    if variable:
        starts = [0]
        while starts[-1] < len(col):
            starts.append(min(len(col), starts[-1] + int(rng.integers(1, 6000))))
        blob = ref.encode(col, starts=starts, regressor="poly")
    else:
        blob = ref.encode(col, fixed_len=700, regressor="poly")
    hd = parse(blob)
    m = hd["m"]
    assert hd["flags"] == (2 | (1 if variable else 0))
    meta = 64 + 32 * m + (8 * (m + 1) if variable else 0)
    coef = -(-meta // 16) * 16
    assert hd["words_off"] == -(-(coef + 16 * m) // 16) * 16
    kinds = blob[64 + 25: 64 + 32 * m: 32]
    assert set(np.unique(kinds)) <= {0, 1} and (kinds == 1).any() and (kinds == 0).any() == variable
    pairs = blob[coef: coef + 16 * m].view(np.float64).reshape(m, 2)
    assert np.all(pairs[kinds == 0] == 0)
    assert np.array_equal(ref.decode_all(blob), col)
    assert len(blob) == -(-(hd["words_off"] + 8 * hd["total_words"]) // 16) * 16


def test_round_trip_and_size(ref):
    for col, L in ((W.cosmos(100_000, 11), 1000), (W.poly_blocks(100_000, 12), 2000),
                   (W.linear_noise(50_000, 13), 1024), (W.lognormal_keys(50_000, 14), 4096)):
        blob = ref.encode(col, fixed_len=L, regressor="poly")
        assert np.array_equal(ref.decode_all(blob), col)
        pos = np.random.default_rng(1).integers(0, len(col), 500)
        assert np.array_equal(ref.random_access(blob, pos), col[pos])
        assert np.array_equal(ref.decode_range(blob, 123, 4567), col[123:4567])
        lo, hi = int(col.min()), int(col.max()) // 2 + 1
        sel = col[(col >= lo) & (col < hi)].astype(object)
        assert ref.filter_sum(blob, lo, hi) == (int(sum(sel)), len(sel))
        # 16 bytes per partition more metadata, never wider residuals
        ls = ref.encode(col, fixed_len=L)
        m = -(-len(col) // L)
        assert len(blob) <= len(ls) + 16 * m + 16


def test_gram_norms_have_closed_forms():
    """The squared norms of the Gram polynomials over t = 0..n-1 (summed
    exactly here) equal the closed forms the GPU fit uses instead of
    summing: (n-1)n(n+1)/3, (n-2)...(n+2)/5, (n-3)...(n+3)/7."""
    for n in list(range(3, 130)) + [1000, 4095, 4096]:
        a = n - 1
        q = [0, 0, 0]
        for t in range(n):
            g1 = 2 * t - a
            g2 = 6 * t * t - 6 * a * t + a * (n - 2)
            g3 = 20 * t ** 3 - 30 * a * t * t + (12 * n * n - 30 * n + 22) * t - a * (n - 2) * (n - 3)
            q[0] += g1 * g1
            q[1] += g2 * g2
            q[2] += g3 * g3
        assert q == [(n - 1) * n * (n + 1) // 3,
                     (n - 2) * (n - 1) * n * (n + 1) * (n + 2) // 5,
                     (n - 3) * (n - 2) * (n - 1) * n * (n + 1) * (n + 2) * (n + 3) // 7], n
