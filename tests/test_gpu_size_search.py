"""GPU parity of the fixed partition size search (section 3.2.1): sampled
costs and whole searches on the GPU, through the C ABI, against the oracle
on the same seeded columns and windows (integers: exact)."""
from __future__ import annotations

import sys

import numpy as np
import pytest

import paper_2306_15374_amd as P
from paper_2306_15374_amd import workloads as W

pytestmark = pytest.mark.gpu


def log(msg: str):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as T
    if not T.cuda.is_available():
        pytest.skip("no GPU")
    return T


@pytest.fixture(scope="module")
def codec(torch):
    c = P.Codec(0)
    yield c
    c.close()


COLUMNS = [
    ("linear_noise", lambda: W.linear_noise(1_000_000, 1)),
    ("lognormal_keys_u64", lambda: W.lognormal_keys(2_000_000, 2)),
    ("lognormal_keys_u32", lambda: W.lognormal_keys(1_000_000, 3).astype(np.uint32)),
    ("piecewise_u32", lambda: W.piecewise_linear(1_000_000, 32, segments=100).astype(np.uint32)),
    ("constant_runs", lambda: W.constant_runs(1_000_000, 33)),
]
LENGTHS = [1, 2, 3, 7, 64, 100, 1000, 1024, 1025, 4096, 4097, 8192, 10_000]


@pytest.mark.parametrize("name,make", COLUMNS, ids=[c[0] for c in COLUMNS])
def test_sampled_costs_match_oracle(torch, codec, ref, name, make):
    col = make()
    starts = W.sample_window_starts(len(col), 10_000, fraction=0.05, seed=7)
    d = torch.from_numpy(col).cuda()
    log(f"[size] costs {name}: n={len(col)} windows={len(starts)}")
    for L in LENGTHS:
        assert codec.fixed_cost(d, starts, 10_000, L) == ref.fixed_cost(col, starts, 10_000, L), L
    for L in (3, 1000, 5000, 10_000):
        got = codec.fixed_cost(d, starts, 10_000, L, regressor="minimax")
        assert got == ref.fixed_cost(col, starts, 10_000, L, regressor="minimax"), L


@pytest.mark.parametrize("name,make", COLUMNS, ids=[c[0] for c in COLUMNS])
def test_search_matches_oracle(torch, codec, ref, name, make):
    col = make()
    starts = W.sample_window_starts(len(col), 10_000, fraction=0.05, seed=8)
    d = torch.from_numpy(col).cuda()
    log(f"[size] search {name}")
    got = codec.size_search(d, starts, 10_000)
    want = ref.size_search(col, starts, 10_000)
    assert got == want


def test_search_with_minimax_and_odd_window(torch, codec, ref):
    col = W.piecewise_linear(500_000, 34, segments=50)
    starts = W.sample_window_starts(len(col), 3_000, fraction=0.05, seed=9)
    d = torch.from_numpy(col).cuda()
    log("[size] minimax search, window 3000")
    assert codec.size_search(d, starts, 3_000, regressor="minimax") == \
        ref.size_search(col, starts, 3_000, regressor="minimax")


def test_window_equal_to_the_column(torch, codec, ref):
    col = W.lognormal_keys(5_000, 4)
    d = torch.from_numpy(col).cuda()
    starts = np.zeros(1, dtype=np.uint64)
    assert codec.size_search(d, starts, 5_000) == ref.size_search(col, starts, 5_000)


def test_size_search_errors(torch, codec):
    col = torch.from_numpy(W.linear_noise(10_000, 5)).cuda()
    ok = np.array([0, 100], dtype=np.uint64)
    cases = [
        (ok, 20_000, 10),                                # window longer than the column
        (np.array([9_000], dtype=np.uint64), 2_000, 10),  # window past the end
        (ok, 1_000, 0),                                  # L = 0
        (ok, 1_000, 1_001),                              # L > window
        (np.zeros(0, dtype=np.uint64), 1_000, 10),       # no windows
    ]
    for starts, window, L in cases:
        st, _ = P.leco_fixed_cost(codec.ctx, col, 10_000, P.LECO_U64, starts, window, L)
        assert st == P.LECO_EINVAL, (starts, window, L)
    st, _ = P.leco_fixed_cost(codec.ctx, col, 10_000, P.LECO_U64, ok, 1_000, 10, regressor=3)
    assert st == P.LECO_EINVAL
    st, *_ = P.leco_size_search(codec.ctx, col, 10_000, P.LECO_U64, ok, 20_000)
    assert st == P.LECO_EINVAL
