"""GPU tests at the shapes of the larger workloads (through the C ABI).

* Three grids beta=50, U=5, dtau in {0.125, 0.1, 0.0625} (L = 400, 500, 800),
  mixed path: replay of the FP64 oracle's flips on sampled chains of each grid
  within 1e-5, and one batched launch of all three grids with 128 chains each.
* Eight grids beta=100, dtau 0.4 .. 0.05 (L = 250 .. 2000), 32 chains per grid,
  mixed path, one batched launch (shortened to one sweep): properties that
  hold at any size (particle-hole symmetry of G(tau), G(0+) = 1/2, bounded
  drift, every chain accounted for), and the multigrid extrapolation onto
  the 4001-point fine grid.
"""
import numpy as np
import pytest

from oracle import bath as OB
from oracle import hfqmc as OH

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch  # noqa: F401  (PyTorch's runtime comes up before the library's)
    import paper_0801_1222_amd as P
    c = P.Context(0)
    yield c
    c.close()


def _codes(ref, L):
    return [sw * L + l for sw, l in ref["flips"]]


@pytest.mark.parametrize("dtau,k", [(0.1, 32), (0.0625, 64)])
def test_three_grid_shape_mixed_replay(ctx, dtau, k):
    import paper_0801_1222_amd as P
    beta, U, seed = 50.0, 5.0, 4
    L = int(round(beta / dtau))
    g0 = OB.bath_to_tau(OB.semicircle_iw(beta, 1.0, 20000), 1.0, beta, L)
    ref = OH.run_chain(g0, U, beta, seed, chain=0, warmup=0, sweeps=1, n_rec=4 * k)
    out = P.hfqmc_solve(ctx, g0, U, beta, dtau, seed, n_chains=1, warmup=0, sweeps=1, n_bins=1,
                        mode="mixed", delay_k=k, replay=[_codes(ref, L)], flip_cap=4000,
                        want_chain=True)
    assert list(out["flips"][0]) == _codes(ref, L)
    got = out["chain_g"][0][0] / out["chain_n"][0][0]
    assert np.abs(got - ref["bins_g"][0]).max() < 1e-5
    assert out["stats"]["n_recomputes"] == ref["n_recomputes"]
    assert 1e-12 < out["stats"]["max_drift"] < 1e-2


def test_three_grid_batched_launch(ctx):
    import paper_0801_1222_amd as P
    beta, U = 50.0, 5.0
    dtaus = [0.125, 0.1, 0.0625]
    Ls = [int(round(beta / d)) for d in dtaus]
    bath = OB.semicircle_iw(beta, 1.0, 20000)
    g0s = [OB.bath_to_tau(bath, 1.0, beta, L) for L in Ls]
    out = P.hfqmc_solve_grids(ctx, Ls, g0s, U, beta, 0, n_chains=128, warmup=1, sweeps=2,
                              mode="mixed", delay_k=64)
    assert Ls == [400, 500, 800]
    for i, L in enumerate(Ls):
        st = out["stats"][i]
        assert st["n_proposed"] == 128 * 3 * L
        assert 0.3 < st["acc_rate"] < 0.8
        assert st["n_bad_ratio"] == 0 and st["n_singular"] == 0
        g = out["g"][i]
        assert abs(g[0] - 0.5) < 1e-5 and abs(g[L] - 0.5) < 1e-5
        assert np.abs(g[1:L] - g[1:L][::-1]).max() < 1e-5
        assert np.all(g > 0) and np.all(g <= 0.5 + 1e-5)


def test_eight_grid_shape_batched_mixed_and_extrapolated(ctx):
    import paper_0801_1222_amd as P
    beta, U, t = 100.0, 5.0, 1.0
    dtaus = [0.4, 0.35, 0.3, 0.25, 0.2, 0.15, 0.1, 0.05]
    bath = OB.semicircle_iw(beta, t, 40000)
    out = P.multigrid_solve(ctx, bath, t * t, U, beta, dtaus, seed=5, n_fine=4001, n_chains=32,
                            warmup=0, sweeps=1, mode="mixed", delay_k=64)
    assert out["Ls"] == [250, 286, 333, 400, 500, 667, 1000, 2000]
    for i, L in enumerate(out["Ls"]):
        st = out["stats"][i]
        assert st["n_proposed"] == 32 * L
        assert st["n_bad_ratio"] == 0 and st["n_singular"] == 0
        assert st["max_drift"] < 5e-2
        g = out["g_grids"][i]
        assert abs(g[0] - 0.5) < 1e-4
        assert np.abs(g[1:L] - g[1:L][::-1]).max() < 1e-4
    g = out["g"]
    assert g.shape == (4001,) and np.all(np.isfinite(g)) and np.all(np.isfinite(out["g_err"]))
    assert np.abs(g - g[::-1]).max() < 1e-4
