"""Pins of the oracle's starting positions for the variable-length split
(section 3.2.2, "Selecting Good Starting Positions").

Linear regressor: for a model of degree k the paper starts partitions in
the segments where the (k+1)-th order deltas are smallest, so here the
second-order deltas dd_k = v_k - 2 v_{k-1} + v_{k-2}: a starting partition
is a maximal run of positions whose |dd| is the column's smallest, with the
three values each such delta spans.

Delta encoding (oracle only, with the Delta-encoding cost): the paper's
recipe of "required bits" (the signed width of each first difference) and
second-order "delta bits" (the change of that width), whose minima start
partitions.  CPU only."""
from __future__ import annotations

import numpy as np
import pytest

import oracle as R

import partition_defs as PD


# ---- linear regressor: second-order deltas ---------------------------------------

@pytest.mark.parametrize("step", [0, 1, 7, 2**20, -3, -(2**33)])
def test_arithmetic_progression_is_one_starting_partition(step):
    """Every second-order delta of a line is zero: one starting partition
    over the whole column."""
    t = np.arange(5000, dtype=np.int64)
    v = (np.int64(2**50) + t * np.int64(step)).astype(np.uint64)
    assert R.starting_partitions(v) == [(0, 5000)]


def test_corner_goes_to_the_later_line():
    """0 1 2 3 4 6 8 10 12 14: slope 1 up to the value 4, slope 2 from it.
    dd_2..dd_9 = 0 0 0 1 0 0 0 0; the runs 2..4 and 6..9 give starting
    partitions [0, 5) and [4, 10), which would share the corner value 4; the
    later keeps it.  The plain split (tau S_M = 4) joins the corner to the
    first line and starts at 5 (d = 2 widens the range: C = 6 * 1 > 4); with
    the starting partitions the second line begins at its corner."""
    v = np.array([0, 1, 2, 3, 4, 6, 8, 10, 12, 14], np.uint64)
    assert R.starting_partitions(v) == [(0, 4), (4, 10)]
    assert list(R.partition_split(v, tau=0.1, sm_bits=40)) == [0, 5, 10]
    assert list(R.partition_split(v, tau=0.1, sm_bits=40, start_positions=True)) == [0, 4, 10]


def test_smallest_second_order_delta_need_not_be_zero():
    """First differences alternating 1, 4: every |dd| is 3, so the whole
    column is one starting partition, and its values join without the cost
    test (at tau = 0 the plain split would cut at every other value)."""
    d = np.tile(np.array([1, 4], np.uint64), 50)
    v = np.concatenate([[np.uint64(7)], np.uint64(7) + np.cumsum(d)]).astype(np.uint64)
    assert R.starting_partitions(v) == [(0, 101)]
    assert list(R.partition_split(v, tau=0.0, sm_bits=320, start_positions=True)) == [0, 101]
    assert len(R.partition_split(v, tau=0.0, sm_bits=320)) - 1 == 51


def test_cubic_has_one_minimum():
    """v = t^3: dd_k = 6k - 6 grows with k, so only position 2 is smallest:
    one starting partition [0, 3)."""
    v = (np.arange(40, dtype=np.uint64) ** np.uint64(3)).astype(np.uint64)
    assert R.starting_partitions(v) == [(0, 3)]


def test_constant_runs_are_their_own_starting_partitions():
    """Runs of one value (lengths 2..9, neighbouring values distinct): dd is
    zero inside runs of length >= 3 (from their third value) and not zero
    at the jumps, so each such run is a starting partition from its first
    to its last value; runs of length 2 are not."""
    rng = np.random.default_rng(4)
    lens = rng.integers(2, 10, 400)
    vals = rng.integers(0, 2**62, 400, dtype=np.uint64)
    vals[1:][vals[1:] == vals[:-1]] += np.uint64(1)
    v = np.repeat(vals, lens)
    run_starts = np.concatenate([[0], np.cumsum(lens)[:-1]])
    expect = [(int(s), int(s + ln)) for s, ln in zip(run_starts, lens) if ln >= 3]
    assert R.starting_partitions(v) == expect


def test_short_columns_have_no_starting_partition():
    for n in (0, 1, 2):
        assert R.starting_partitions(np.arange(n, dtype=np.uint64)) == []


@pytest.mark.parametrize("seed", range(12))
@pytest.mark.parametrize("dtype", [np.uint32, np.uint64])
def test_starting_partitions_equal_python_definition(seed, dtype):
    """Recomputed in Python from the second-order deltas on random columns:
    noise, lines with noise, runs, and values near both ends of the range."""
    rng = np.random.default_rng(seed)
    n = int(rng.integers(3, 3000))
    top = 2**32 - 1 if dtype == np.uint32 else 2**64 - 1
    kind = seed % 4
    if kind == 0:
        v = rng.integers(0, 16, n, dtype=np.uint64)
    elif kind == 1:
        v = np.arange(n, dtype=np.uint64) * np.uint64(3) + rng.integers(0, 3, n, dtype=np.uint64)
    elif kind == 2:
        v = np.repeat(rng.integers(0, 1000, n, dtype=np.uint64), rng.integers(1, 6, n))[:n]
    else:
        v = rng.integers(0, top, n, dtype=np.uint64, endpoint=True)
        v[::3] = np.uint64(top) - rng.integers(0, 4, len(v[::3]), dtype=np.uint64)
        v[1::3] = rng.integers(0, 4, len(v[1::3]), dtype=np.uint64)
    v = v.astype(dtype)
    assert R.starting_partitions(v) == PD.starting_partitions(v)


def test_greedy_with_starting_positions_merges_its_own_split():
    rng = np.random.default_rng(10)
    t = np.arange(8000)
    v = (t * 3 + rng.integers(0, 1 << (t // 1000 + 1), 8000)).astype(np.uint64)
    split = R.partition_split(v, tau=0.05, sm_bits=320, start_positions=True)
    full = R.partition_greedy(v, tau=0.05, sm_bits=320, start_positions=True)
    assert list(R.partition_merge(v, split)) == list(full)
    assert set(int(a) for a, _ in R.starting_partitions(v)) <= set(int(s) for s in split)


def test_split_without_starting_positions_is_unchanged():
    rng = np.random.default_rng(9)
    v = np.sort(rng.integers(0, 2**40, 5000, dtype=np.uint64))
    plain = R.partition_split(v, tau=0.1, sm_bits=320)
    both = R.partition_greedy(v, tau=0.1, sm_bits=320)
    assert set(both) <= set(plain)
    assert list(R.partition_merge(v, plain)) == list(both)


# ---- Delta encoding: required bits and delta bits ---------------------------------

@pytest.mark.parametrize("v0", [0, 10, 28, 32, 100, 2**40])
def test_delta_figure_segment_is_a_starting_partition(v0):
    """The Delta-encoding figure grows the segment {30, 31, 32}: its two
    differences are 1 and 1 (2 signed bits each, zero delta bits), so the
    segment starts a partition at its first value whatever precedes it,
    unless that value is also one step away from 30 (then the run of zero
    delta bits, and the starting partition, begin one value earlier)."""
    v = np.array([v0, 30, 31, 32, 29, 49], np.uint64)
    assert list(R.start_positions_delta(v)) == [1]


@pytest.mark.parametrize("v0", [29, 31])
def test_delta_figure_segment_extends_back_one_value(v0):
    v = np.array([v0, 30, 31, 32, 29, 49], np.uint64)
    assert list(R.start_positions_delta(v)) == [0]


def test_delta_smallest_delta_bits_need_not_be_zero():
    """Differences alternating between widths 2 and 4 bits (1, 4, 1, 4, ...):
    every delta bit is 2, the column's smallest: one starting partition."""
    d = np.tile(np.array([1, 4], np.uint64), 500)
    v = np.concatenate([[np.uint64(100)], np.uint64(100) + np.cumsum(d)]).astype(np.uint64)
    assert list(R.start_positions_delta(v)) == [0]


def test_delta_short_columns_have_none():
    for n in (0, 1, 2):
        assert len(R.start_positions_delta(np.arange(n, dtype=np.uint64))) == 0
