"""Drift and statistical parity of the mixed-precision path at the headline shape.

The mixed path (FP32 flush products, FP64 ratios, acceptance and recompute)
is not flip-identical to the FP64 method once it runs free, so beyond the
replay tests it is checked here as a sampler:

  * the drift statistics: the G(tau)-level drift (max_drift_gtau) vanishes on
    the FP64 paths and stays below the elementwise drift on the mixed path;
    on the oracle's own flips and flush points (every recompute sampled) the
    mixed path's drift is that of the oracle's FP32 flush emulation within a
    factor of 3 (the two factorizations of the rank-m product round alike);
  * free-running statistics at beta = 40, U = 4.5, L = 400 with k = 64 and a
    recompute every 256 accepted flips: D and G(tau_k) agree with an
    independent FP64 run (the delayed FP64 path, flip for flip the oracle)
    within 3 sigma of the combined error, at most 1 % of the points beyond
    3 sigma and none beyond 5 sigma.
"""
import numpy as np
import pytest

from oracle import bath as OB
from oracle import hfqmc as OH
from stat_checks import compare_3sigma

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch  # noqa: F401  (PyTorch's runtime comes up before the library's)
    import paper_0801_1222_amd as P
    c = P.Context(0)
    yield c
    c.close()


def _bath(beta, L, t=1.0):
    return OB.bath_to_tau(OB.semicircle_iw(beta, t, 20000), t * t, beta, L)


def _codes(ref, L):
    return [sw * L + l for sw, l in ref["flips"]]


@pytest.mark.parametrize("mode,k", [("rank1", 0), ("delayed", 32)])
def test_gtau_drift_vanishes_on_fp64_paths(ctx, mode, k):
    import paper_0801_1222_amd as P
    beta, U, L = 13.0, 4.8, 130
    out = P.hfqmc_solve(ctx, _bath(beta, L), U, beta, 0.1, 5, n_chains=8, warmup=2, sweeps=6,
                        mode=mode, delay_k=k, recompute_every=50, drift_every=1)
    st = out["stats"]
    assert st["n_recomputes"] >= 8 * 10
    assert st["max_drift"] < 1e-10
    assert 0.0 <= st["max_drift_gtau"] < 1e-12
    assert st["max_drift_gtau"] <= st["max_drift"]


def test_mixed_gtau_drift_below_elementwise(ctx):
    import paper_0801_1222_amd as P
    beta, U, L = 40.0, 4.5, 400
    out = P.hfqmc_solve(ctx, _bath(beta, L), U, beta, 0.1, 0, n_chains=32, warmup=0, sweeps=4,
                        mode="mixed", delay_k=64, drift_every=1)
    st = out["stats"]
    assert st["n_recomputes"] >= 32 * 2
    assert 0.0 < st["max_drift_gtau"] <= st["max_drift"]
    # the estimator averages L entries per lag: far below the elementwise drift
    assert st["max_drift_gtau"] < 1e-4


def test_mixed_drift_matches_oracle_fp32_emulation(ctx):
    """Same flips (the FP64 oracle's, replayed) and the same flush points on both
    sides: a flush at k pending, before every recompute, at each sweep end."""
    import paper_0801_1222_amd as P
    beta, U, L, k, sweeps = 40.0, 4.5, 400, 64, 3
    g0 = _bath(beta, L)
    chains = [0, 1, 2, 3]
    refs = [OH.run_chain(g0, U, beta, 0, chain=c, warmup=0, sweeps=sweeps, n_rec=4 * k)
            for c in chains]
    emu = [OH.run_chain(g0, U, beta, 0, chain=c, warmup=0, sweeps=sweeps, n_rec=4 * k,
                        delay_k=k, flush_fp32=True, replay=set(r["flips"]))
           for c, r in zip(chains, refs)]
    out = P.hfqmc_solve(ctx, g0, U, beta, 0.1, 0, n_chains=len(chains), warmup=0, sweeps=sweeps,
                        mode="mixed", delay_k=k, replay=[_codes(r, L) for r in refs],
                        flip_cap=20000, want_chain=True, drift_every=1)
    for c in chains:
        assert list(out["flips"][c]) == _codes(refs[c], L)
    n_rec = sum(e["n_recomputes"] for e in emu)
    assert out["stats"]["n_recomputes"] == n_rec and n_rec >= 8
    gpu = float(np.max(out["chain_drift"]))
    orc = max(e["max_drift"] for e in emu)
    assert orc / 3.0 <= gpu <= 3.0 * orc, (gpu, orc)


def test_mixed_free_running_matches_fp64(ctx):
    """256 chains x (100 + 1000) sweeps in each mode, independent seeds."""
    import paper_0801_1222_amd as P
    beta, U, L = 40.0, 4.5, 400
    g0 = _bath(beta, L)
    kw = dict(n_chains=256, warmup=100, sweeps=1000, delay_k=64)
    mx = P.hfqmc_solve(ctx, g0, U, beta, 0.1, 0, mode="mixed", **kw)
    fp = P.hfqmc_solve(ctx, g0, U, beta, 0.1, 1 << 32, mode="delayed", **kw)
    assert mx["stats"]["recompute_every"] == 256 and fp["stats"]["recompute_every"] == 256
    assert mx["stats"]["n_bad_ratio"] == 0
    # G(0+) = G(beta-) = 1/2 exactly at half filling: the interior lags
    compare_3sigma(mx["g"][1:L], mx["g_err"][1:L], fp["g"][1:L], fp["g_err"][1:L])
    z = abs(mx["D"] - fp["D"]) / np.hypot(mx["D_err"], fp["D_err"])
    assert z < 3.0, (mx["D"], fp["D"], z)


def test_mixed_free_running_matches_fp64_long_grid(ctx):
    """L = 1000 (beta = 100, dtau = 0.1), the long-grid instantiation with the LU
    panel in the workspace: mixed against FP64 delayed, 256 chains x (10 + 40)
    sweeps each, independent seeds; D and G(tau) by the 3-sigma rule."""
    import paper_0801_1222_amd as P
    beta, U, L = 100.0, 4.8, 1000
    g0 = _bath(beta, L)
    kw = dict(n_chains=256, warmup=10, sweeps=40, delay_k=64)
    mx = P.hfqmc_solve(ctx, g0, U, beta, 0.1, 7, mode="mixed", **kw)
    fp = P.hfqmc_solve(ctx, g0, U, beta, 0.1, 7 + (1 << 32), mode="delayed", **kw)
    assert mx["stats"]["n_bad_ratio"] == 0 and fp["stats"]["n_bad_ratio"] == 0
    assert mx["stats"]["lu_panel"] in (16, 32)       # the matrix-core LU, panel in the workspace
    compare_3sigma(mx["g"][1:L], mx["g_err"][1:L], fp["g"][1:L], fp["g_err"][1:L])
    z = abs(mx["D"] - fp["D"]) / np.hypot(mx["D_err"], fp["D_err"])
    assert z < 3.0, (mx["D"], fp["D"], z)
