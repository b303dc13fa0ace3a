"""Pins of the oracle's fixed partition size search (section 3.2.1): the
sampled cost against closed forms and the blob format, the search against
synthetic cost curves with known minima and against brute force.  CPU
only."""
from __future__ import annotations

import numpy as np
import pytest

from paper_2306_15374_amd import workloads as W


def test_cost_of_linear_columns_is_records_only(ref):
    """An arithmetic progression fits with width 0 in every partition, so
    the cost is 32 bytes per partition: 32 * k * ceil(window / L)."""
    col = (np.arange(50_000, dtype=np.uint64) * np.uint64(13) + np.uint64(5))
    starts = [0, 17, 40_000]
    for L in (1, 7, 64, 1000, 4096, 9_999, 10_000):
        assert ref.fixed_cost(col, starts, 10_000, L) == 32 * 3 * -(-10_000 // L)


def test_cost_of_alternating_bits(ref):
    """v_t = t mod 2: one or two values lie on a line (width 0); three or
    more alternating values fit no line exactly, so the constant model's
    width 1 is stored."""
    col = (np.arange(20_000) % 2).astype(np.uint32)
    for L in (1, 2, 3, 64, 65, 1000):
        want = 0
        for p in range(0, 5000, L):
            ln = min(L, 5000 - p)
            want += 32 + 8 * -(-(ln * (1 if ln > 2 else 0)) // 64)
        assert ref.fixed_cost(col, [100, 7000], 5000, L) == 2 * want


@pytest.mark.parametrize("regressor", ["ls", "minimax"])
def test_cost_equals_record_and_word_bytes_of_the_windows_blobs(ref, regressor):
    """Encoding each window on its own with fixed partitions of L gives m
    records and total_words words (header fields): the cost is
    sum(32 m + 8 total_words)."""
    col = W.lognormal_keys(300_000, 2)
    rng = np.random.default_rng(5)
    starts = rng.integers(0, len(col) - 3000, 6)
    for L in (1, 10, 300, 1024, 3000):
        want = 0
        for s in starts:
            blob = ref.encode(col[s:s + 3000], fixed_len=L, regressor=regressor)
            hdr = blob[:64].view(np.uint64)
            want += 32 * int(hdr[2]) + 8 * int(hdr[7])
        assert ref.fixed_cost(col, starts, 3000, L, regressor=regressor) == want


@pytest.mark.parametrize("center", [1, 2, 3, 100, 300, 511, 512, 513, 777, 1000])
def test_search_finds_the_minimum_of_a_convex_curve(ref, center):
    """On a strictly convex cost the exponential phase brackets the minimum
    within a factor of two and every halving step keeps it within twice the
    step, so the last step (s = 1) lands on it."""
    r = ref.size_search_fn(1000, lambda L: (L - center) ** 2 * 1000 + 7)
    assert r["L"] == center and r["cost"] == 7


def test_search_trace_by_hand(ref):
    """cost(L) = |L - 300| + 10^6 on [1, 1000]: the exponential phase
    evaluates 1 .. 512 (512 costs more than 256) and keeps 256 (cost
    10^6 + 44); the back search with s = 128 compares 128 (already
    evaluated, not traced again) and 384, both dearer, so it stays; with s = 64 it tries 192 and 320 and moves to 320 (10^6 +
    20), a decline of 24 / (10^6 + 44) < 0.01%, so it stops there."""
    r = ref.size_search_fn(1000, lambda L: abs(L - 300) + 10**6)
    assert [L for L, _ in r["trace"]] == [1, 2, 4, 8, 16, 32, 64, 128, 256, 512, 384, 192, 320]
    assert r["L"] == 320 and r["cost"] == 10**6 + 20
    # the window itself is tried when it is not a power of two
    r = ref.size_search_fn(700, lambda L: 10**9 - L)
    assert [L for L, _ in r["trace"]][:11] == [1, 2, 4, 8, 16, 32, 64, 128, 256, 512, 700]
    assert r["L"] == 700


def test_search_agrees_with_its_costs(ref):
    """Every traced cost is the sampled cost of its L, the result is the
    cheapest traced L, and the exponential phase doubles until the first
    increase."""
    col = W.lognormal_keys(2_000_000, 2)
    starts = np.random.default_rng(9).integers(0, len(col) - 8192, 8)
    r = ref.size_search(col, starts, 8192)
    costs = dict(r["trace"])
    for L, c in r["trace"][:6]:
        assert ref.fixed_cost(col, starts, 8192, L) == c
    assert r["cost"] == ref.fixed_cost(col, starts, 8192, r["L"]) == min(costs.values())
    exp = [L for L, _ in r["trace"]]
    k = 0
    while k + 1 < len(exp) and exp[k + 1] == 2 * exp[k]:
        k += 1
    assert exp[0] == 1 and costs[exp[k]] > costs[exp[k - 1]]


def test_search_on_a_u_shaped_column_matches_brute_force(ref):
    """A linear column with noise and a slow bend: short partitions pay
    records, long ones pay the bend in residual width, so the cost is
    U-shaped in L; on this seeded column the search reaches the brute-force
    optimum over every L in [1, 600]."""
    rng = np.random.default_rng(10)
    t = np.arange(200_000, dtype=np.float64)
    col = (1e6 + 5 * t + 2e-4 * (t % 20_000) ** 2 + rng.integers(0, 16, len(t))).astype(np.uint64)
    starts = rng.integers(0, len(col) - 600, 5)
    costs = [ref.fixed_cost(col, starts, 600, L) for L in range(1, 601)]
    best = int(np.argmin(costs)) + 1
    r = ref.size_search(col, starts, 600)
    assert costs[best - 1] < costs[0] and costs[best - 1] < costs[-1]  # U-shaped
    assert r["cost"] == costs[best - 1]


def test_size_search_rejects_bad_arguments(ref):
    import oracle
    col = W.linear_noise(1000, 1)
    with pytest.raises(oracle.OracleError):
        ref.fixed_cost(col, [500], 600, 10)   # window past the end
    with pytest.raises(oracle.OracleError):
        ref.fixed_cost(col, [0], 600, 601)    # L > window
    with pytest.raises(oracle.OracleError):
        ref.size_search(col, [], 600)         # no window
