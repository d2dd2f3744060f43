"""CPU checks of the chain-split planner behind HFQMC_FLAG_BALANCE.

The planner models a batched launch as units (grid, chain) of cost
(warmup + sweeps_i) L_i^3 taken longest first by P workgroups.  Its spans are
checked against an independent longest-first simulation written here, its
choice against an exhaustive search over the split factors on small cases, and
its constraints (power of two, divides sweeps, at least n_bins sweeps per
chain) directly.  Host logic only: no GPU.
"""
import heapq
import itertools

import numpy as np
import pytest


def _lpt(costs, p):
    """Longest-processing-time-first list scheduling on p identical workers."""
    costs = sorted(costs, reverse=True)
    p = max(1, min(p, len(costs)))
    fin = [0.0] * p
    span = 0.0
    for c in costs:
        t = heapq.heappop(fin) + c
        span = max(span, t)
        heapq.heappush(fin, t)
    return span


def _span(Ls, n_chains, warmup, sweeps, factors, p):
    costs = []
    for L, f in zip(Ls, factors):
        costs += [(warmup + sweeps // f) * float(L) ** 3] * (n_chains * f)
    return _lpt(costs, p)


def _plan(*a):
    import paper_0801_1222_amd as P
    return P.hfqmc_plan_balance(*a)


def test_even_grids_are_not_split():
    # every workgroup busy and equal units: a split only adds warm-ups
    r = _plan([400, 400, 400, 400], 64, 100, 1000, 1, 256)
    assert r["factor"] == [1, 1, 1, 1]
    assert r["span_after"] == r["span_before"]


def test_eight_grid_cycle_splits_the_long_grids():
    Ls = [250, 286, 333, 400, 500, 667, 1000, 2000]
    r = _plan(Ls, 32, 100, 1000, 1, 256)
    f = r["factor"]
    assert f[-1] >= 4 and f[0] == 1
    assert all(a <= b for a, b in zip(f, f[1:]))        # longer grids split at least as much
    assert r["span_before"] == pytest.approx(_span(Ls, 32, 100, 1000, [1] * 8, 256), rel=1e-12)
    assert r["span_after"] == pytest.approx(_span(Ls, 32, 100, 1000, f, 256), rel=1e-12)
    # the unsplit launch is as long as one L = 2000 chain; the plan is at least 3x shorter
    assert r["span_before"] == pytest.approx(1100 * 2000.0 ** 3, rel=1e-12)
    assert r["span_after"] < r["span_before"] / 3


def test_single_grid_few_chains_fills_the_device():
    # 32 chains on 256 workgroups: f = 8 gives one chain of 100 + 125 sweeps per workgroup
    r = _plan([2000], 32, 100, 1000, 1, 256)
    assert r["factor"] == [8]
    assert r["span_after"] == pytest.approx(225 * 2000.0 ** 3, rel=1e-12)


def _cases():
    rng = np.random.default_rng(11)
    fixed = [([100, 200, 400], 4, 10, 64, 32), ([60, 120, 240], 8, 50, 128, 48),
             ([300, 310, 900], 2, 5, 32, 16)]
    rand = []
    for _ in range(12):
        n = int(rng.integers(2, 4))
        Ls = sorted(int(x) for x in rng.integers(20, 1000, size=n))
        rand.append((Ls, int(rng.integers(1, 9)), int(rng.integers(0, 60)), 64,
                     int(rng.integers(4, 65))))
    return fixed + rand


@pytest.mark.parametrize("Ls,n_chains,warmup,sweeps,p", _cases())
def test_plan_matches_exhaustive_search(Ls, n_chains, warmup, sweeps, p):
    r = _plan(Ls, n_chains, warmup, sweeps, 1, p)
    combos = itertools.product([1, 2, 4, 8, 16, 32, 64], repeat=len(Ls))
    best = min(_span(Ls, n_chains, warmup, sweeps, fs, p) for fs in combos)
    got = _span(Ls, n_chains, warmup, sweeps, r["factor"], p)
    assert got == pytest.approx(r["span_after"], rel=1e-12)
    assert got <= r["span_before"] * (1 + 1e-12)
    # within 5 % of the best split over every factor combination
    assert got <= 1.05 * best, (r["factor"], got / best)


def test_split_respects_sweeps_and_bins():
    # sweeps = 12: at most f = 4 (12 / 8 is not whole)
    r = _plan([2000], 1, 0, 12, 1, 256)
    assert r["factor"] == [4]
    # an odd sweep count cannot be split
    assert _plan([2000], 1, 0, 15, 1, 256)["factor"] == [1]
    # n_bins = 4 of 16 sweeps: f <= 4
    assert _plan([2000], 1, 0, 16, 4, 256)["factor"] == [4]
    # f never exceeds 64
    assert _plan([2000], 1, 0, 1 << 12, 1, 4096)["factor"] == [64]


def test_large_launches_are_left_unsplit():
    # more than 8192 chains in all: not planned
    r = _plan([250, 2000], 4097, 10, 96, 1, 256)
    assert r["factor"] == [1, 1] and r["span_before"] == 0.0 and r["span_after"] == 0.0
    assert _plan([250, 2000], 4096, 10, 96, 1, 256)["span_before"] > 0.0
    # just below the limit the long grid still splits
    assert _plan([2000], 8, 10, 96, 1, 256)["factor"][0] > 1


def test_plan_argument_errors():
    import paper_0801_1222_amd as P
    bad = [([], 1, 0, 10, 1, 8), ([1], 1, 0, 10, 1, 8), ([100], 0, 0, 10, 1, 8),
           ([100], 1, -1, 10, 1, 8), ([100], 1, 0, 0, 1, 8), ([100], 1, 0, 10, 11, 8),
           ([100], 1, 0, 10, 1, 0)]
    for a in bad:
        with pytest.raises(P.HFQMCError) as e:
            _plan(*a)
        assert e.value.code == -1
