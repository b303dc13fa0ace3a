"""Pins of the oracle's starting positions for the variable-length split
(section 3.2.2, "Selecting Good Starting Positions", and the partitioning
figure), under the reading that the required bits of a first difference are
its signed width and the delta bits are the change of that width between
neighbouring differences; a starting partition is a maximal run of positions
with the column's smallest delta bits, extended back to its first three
values.  CPU only."""
from __future__ import annotations

import numpy as np
import pytest

import oracle as R


@pytest.mark.parametrize("v0", [0, 10, 28, 32, 100, 2**40])
def test_figure_segment_is_a_starting_partition(v0):
    """The figure's worked example grows the segment {30, 31, 32}: its two
    differences are 1 and 1 (2 signed bits each, zero delta bits), so the
    segment starts a partition at its first value whatever precedes it,
    unless that value is also one step away from 30 (then the run of zero
    delta bits, and the starting partition, begin one value earlier)."""
    v = np.array([v0, 30, 31, 32, 29, 49], np.uint64)
    assert list(R.start_positions(v)) == [1]


@pytest.mark.parametrize("v0", [29, 31])
def test_figure_segment_extends_back_one_value(v0):
    v = np.array([v0, 30, 31, 32, 29, 49], np.uint64)
    assert list(R.start_positions(v)) == [0]


@pytest.mark.parametrize("step", [0, 1, 7, 2**20, -3, -(2**33)])
def test_arithmetic_progression_is_one_starting_partition(step):
    """Every difference equal: every delta bit is zero, one run from the
    first value."""
    t = np.arange(5000, dtype=np.int64)
    v = (np.int64(2**50) + t * np.int64(step)).astype(np.uint64)
    assert list(R.start_positions(v)) == [0]


def test_smallest_delta_bits_need_not_be_zero():
    """Differences alternating between widths 2 and 4 bits (1, 4, 1, 4, ...):
    every delta bit is 2, the column's smallest, so the whole column is one
    starting partition."""
    d = np.tile(np.array([1, 4], np.uint64), 500)
    v = np.concatenate([[np.uint64(100)], np.uint64(100) + np.cumsum(d)]).astype(np.uint64)
    assert list(R.start_positions(v)) == [0]


def test_constant_runs_start_where_runs_of_three_or_more_begin():
    """Runs of one value (lengths 2..9, neighbouring values distinct): the
    differences inside a run are 0 (1 signed bit) and the jumps between runs
    are wider, so the zero delta bits lie inside runs of length >= 3 and each
    such run starts a partition at its first value; runs of length 2 do not."""
    rng = np.random.default_rng(4)
    lens = rng.integers(2, 10, 400)
    vals = rng.integers(0, 2**62, 400, dtype=np.uint64)
    vals[1:][vals[1:] == vals[:-1]] += np.uint64(1)
    v = np.repeat(vals, lens)
    run_starts = np.concatenate([[0], np.cumsum(lens)[:-1]])
    expect = [int(s) for s, ln in zip(run_starts, lens) if ln >= 3]
    assert list(R.start_positions(v)) == expect


def test_short_columns_have_no_starting_partition():
    for n in (0, 1, 2):
        assert len(R.start_positions(np.arange(n, dtype=np.uint64))) == 0


@pytest.mark.parametrize("seed", [1, 2, 3])
@pytest.mark.parametrize("dtype", [np.uint32, np.uint64])
def test_split_restarts_at_each_starting_partition(seed, dtype):
    """With starting positions the split is the plain split run separately on
    each stretch between consecutive starting positions: the inclusion test
    is unchanged, a partition merely also begins at every such position."""
    rng = np.random.default_rng(seed)
    n = 6000
    t = np.arange(n)
    # smooth stretches, noisy stretches and a jump every 700 values
    v = (1000 + 5 * t + np.where((t // 350) % 2 == 0, 0, rng.integers(0, 5000, n))
         + (t // 700) * 100000).astype(dtype)
    forced = [int(p) for p in R.start_positions(v)]
    assert len(forced) > 3
    got = R.partition_split(v, tau=0.05, sm_bits=320, start_positions=True)
    cuts = sorted(set([0] + forced + [n]))
    expect = []
    for a, b in zip(cuts[:-1], cuts[1:]):
        expect += [a + int(s) for s in R.partition_split(v[a:b], tau=0.05, sm_bits=320)[:-1]]
    assert list(got) == expect + [n]
    assert set(forced) <= set(int(s) for s in got)


def test_split_without_starting_positions_is_unchanged():
    rng = np.random.default_rng(9)
    v = np.sort(rng.integers(0, 2**40, 5000, dtype=np.uint64))
    plain = R.partition_split(v, tau=0.1, sm_bits=320)
    both = R.partition_greedy(v, tau=0.1, sm_bits=320, max_rounds=0)
    assert set(both) <= set(plain)
    merged = R.partition_merge(v, plain)
    assert list(merged) == list(both)


def test_greedy_with_starting_positions_merges_its_own_split():
    rng = np.random.default_rng(10)
    t = np.arange(8000)
    v = (t * 3 + rng.integers(0, 1 << (t // 1000 + 1), 8000)).astype(np.uint64)
    split = R.partition_split(v, tau=0.05, sm_bits=320, start_positions=True)
    full = R.partition_greedy(v, tau=0.05, sm_bits=320, start_positions=True)
    assert list(R.partition_merge(v, split)) == list(full)
