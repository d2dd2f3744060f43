"""The largest grids: the last L the LDS staging of the LU admits runs, the
next one is refused before any device work.

At L = 3072 (beta = 153.6, dtau = 0.05; one sweep of two chains, mixed path,
the LU on 8-wide panels of an |S| <= 1536 system and L-row reference solves)
the properties that hold at any size: G(0+) + G(beta-) = 1, G(tau) = G(beta - tau)
for the half-filled bath (to the mixed path's rounding), finite results, the
G(tau)-level drift far below the elementwise one.  L = 3200 needs more LDS for
its reference solve than a workgroup has: HFQMC_EUNSUPPORTED.
"""
import numpy as np
import pytest

from oracle import bath as OB

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch  # noqa: F401  (PyTorch's runtime comes up before the library's)
    import paper_0801_1222_amd as P
    c = P.Context(0)
    yield c
    c.close()


def test_largest_grid_runs(ctx):
    import paper_0801_1222_amd as P
    beta, U, L = 153.6, 4.0, 3072
    g0 = OB.bath_to_tau(OB.semicircle_iw(beta, 1.0, 20000), 1.0, beta, L)
    out = P.hfqmc_solve(ctx, g0, U, beta, beta / L, 5, n_chains=2, warmup=0, sweeps=1,
                        mode="mixed", delay_k=64, n_bins=1, drift_every=1)
    g, st = out["g"], out["stats"]
    assert np.all(np.isfinite(g)) and np.isfinite(out["D"])
    assert abs(g[0] + g[L] - 1.0) < 1e-12
    assert np.abs(g[1:L] - g[L - 1:0:-1]).max() < 1e-8
    assert st["n_bad_ratio"] == 0 and st["n_singular"] == 0 and st["n_recomputes"] >= 4
    assert 0.0 < st["max_drift_gtau"] < 1e-6 and st["max_drift"] < 1e-3
    assert 0.05 < out["D"] < 0.25


def test_grid_beyond_the_lds_capacity_is_refused(ctx):
    import paper_0801_1222_amd as P
    beta, L = 160.0, 3200
    g0 = OB.bath_to_tau(OB.semicircle_iw(beta, 1.0, 4000), 1.0, beta, L)
    with pytest.raises(P.HFQMCError) as e:
        P.hfqmc_solve(ctx, g0, 4.0, beta, beta / L, 1, n_chains=1, warmup=0, sweeps=1,
                      mode="delayed", delay_k=32, n_bins=1)
    assert e.value.code == -6 and "LDS" in str(e.value)
