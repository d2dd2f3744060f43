"""The mixed-precision path against the oracle's own Monte Carlo estimates.

tests/golden/oracle_mc_*.txt hold estimates of the FP64 oracle (written by
make_golden_mc.py, seeds disjoint from the ones used here), so the GPU run is
an independent sample of the same fixed-dtau expectation: D and G(tau) must
agree within 3 sigma of the combined error (at most 1 % of the points beyond
3 sigma, none beyond 5 sigma).
"""
import os

import numpy as np
import pytest

from oracle import bath as OB
from stat_checks import compare_3sigma, read_fixture

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def ctx():
    import torch  # noqa: F401  (PyTorch's runtime comes up before the library's)
    import paper_0801_1222_amd as P
    c = P.Context(0)
    yield c
    c.close()


def test_mixed_headline_shape_matches_oracle_monte_carlo(ctx):
    """beta = 40, U = 4.5, L = 400: mixed path, k = 64, recompute every 256,
    256 chains x (200 + 1000) sweeps against the oracle's 64 chains x (200 + 800)."""
    import paper_0801_1222_amd as P
    fx = read_fixture(os.path.join(HERE, "golden", "oracle_mc_b40_u45_L400.txt"))
    beta, U, L = 40.0, 4.5, 400
    og = np.array(fx["G"])
    assert og.shape == (L + 1, 3)
    g0 = OB.bath_to_tau(OB.semicircle_iw(beta, 1.0, 20000), 1.0, beta, L)
    out = P.hfqmc_solve(ctx, g0, U, beta, 0.1, 0, n_chains=256, warmup=200, sweeps=1000,
                        mode="mixed", delay_k=64)
    assert out["stats"]["recompute_every"] == 256
    compare_3sigma(out["g"][1:L], out["g_err"][1:L], og[1:L, 1], og[1:L, 2])
    (d, de), = fx["D"]
    assert abs(out["D"] - d) < 3.0 * np.hypot(out["D_err"], de), (out["D"], d)


def test_mixed_multigrid_matches_oracle_monte_carlo(ctx):
    """Seven grids beta = 20, U = 4.8, L = 50 .. 160, 64 chains x (200 + 2000) sweeps
    per grid: the mixed path's multigrid step against the oracle's (FP64 rank-1
    chains, independent seeds): every grid's G(tau_k) and D, the dtau -> 0
    extrapolated G on the 200-point fine grid and the extrapolated D."""
    import paper_0801_1222_amd as P
    fx = read_fixture(os.path.join(HERE, "golden", "oracle_mc_b20_u48_mg7.txt"))
    beta, U, t = 20.0, 4.8, 1.0
    dtaus = [0.4, 1 / 3, 2 / 7, 0.25, 0.2, 1 / 6, 0.125]
    bath = P.bethe_semicircle_bath(beta, t, 20000)
    out = P.multigrid_solve(ctx, bath, t * t, U, beta, dtaus, 0, n_fine=200, n_chains=64,
                            warmup=200, sweeps=2000, mode="mixed", delay_k=32)
    assert out["Ls"] == [50, 60, 70, 80, 100, 120, 160]
    gg = np.array(fx["GG"])
    gd = np.array(fx["GD"])
    for i, L in enumerate(out["Ls"]):
        rows = gg[gg[:, 0] == i]
        assert rows.shape[0] == L + 1 and int(gd[i, 1]) == L
        st = out["stats"][i]
        assert st["recompute_every"] == 128 and st["n_bad_ratio"] == 0
        g = out["g_grids"][i]
        # multigrid_solve returns the grids' G(tau) without their errors: the two runs
        # have the same statistics per grid, so the oracle's error stands for both
        compare_3sigma(g[1:L], rows[1:L, 3], rows[1:L, 2], rows[1:L, 3])
        assert abs(out["D_grids"][i] - gd[i, 2]) < 3.0 * np.hypot(out["D_err_grids"][i], gd[i, 3])
    f = np.array(fx["F"])
    assert f.shape == (200, 3)
    # interior fine points (tau = 0+ and beta- are exactly 1/2)
    compare_3sigma(out["g"][1:-1], out["g_err"][1:-1], f[1:-1, 1], f[1:-1, 2])
    (d, de), = fx["D"]
    assert abs(out["D"] - d) < 3.0 * np.hypot(out["D_err"], de), (out["D"], d)
