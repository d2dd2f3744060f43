"""The largest grids.

L = 4096 is the largest grid the library accepts.  Its uniform-field reference
solves (4096-row systems) keep their LU panel in the workspace, the chains'
reduced recomputes (|S| <= 2048 rows) run on 4-wide LDS panels.  One sweep of
two chains on the mixed path (beta = 204.8, dtau = 0.05, a recompute every 1024
accepted flips) is checked by the properties that hold at any size:
G(0+) + G(beta-) = 1, G(tau) = G(beta - tau) for the half-filled bath (to the
mixed path's rounding), finite results, the G(tau)-level drift far below the
elementwise one.  On the FP64 delayed path the final G of a sweep is compared
with the exact solution of the Dyson equation for the final field (the
oracle's dense solve; the field from the initial Philox draw and the flip
log).  The full-size recompute (HFQMC_FLAG_DIRECT_RECOMPUTE) stages
an L-row panel in LDS and stops at L = 3092: L = 3200 is refused with
HFQMC_EUNSUPPORTED before any device work.
"""
import numpy as np
import pytest

from oracle import bath as OB
from oracle import hfqmc as OH
from oracle import philox

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
    beta, U, L = 204.8, 4.0, 4096
    g0 = OB.bath_to_tau(OB.semicircle_iw(beta, 1.0, 20000), 1.0, beta, L)
    out = P.hfqmc_solve(ctx, g0, U, beta, beta / L, 5, n_chains=2, warmup=0, sweeps=1,
                        mode="mixed", delay_k=64, recompute_every=1024, n_bins=1, drift_every=1)
    g, st = out["g"], out["stats"]
    assert np.all(np.isfinite(g)) and np.isfinite(out["D"])
    assert abs(g[0] + g[L] - 1.0) < 1e-12
    assert np.abs(g[1:L] - g[L - 1:0:-1]).max() < 1e-7
    assert st["n_bad_ratio"] == 0 and st["n_singular"] == 0 and st["n_recomputes"] >= 4
    assert 0.0 < st["max_drift_gtau"] < 1e-5 and st["max_drift"] < 1e-2
    assert 0.05 < out["D"] < 0.25


def test_largest_grid_final_green_is_exact(ctx):
    import paper_0801_1222_amd as P
    beta, U, L, seed = 204.8, 4.0, 4096, 2
    g0 = OB.bath_to_tau(OB.semicircle_iw(beta, 1.0, 20000), 1.0, beta, L)
    out = P.hfqmc_solve(ctx, g0, U, beta, beta / L, seed, n_chains=1, warmup=0, sweeps=1,
                        mode="delayed", delay_k=64, recompute_every=1024, n_bins=1,
                        flip_cap=2 * L, want_green=True)
    st = out["stats"]
    assert st["n_recomputes"] >= 3 and st["max_drift"] < 1e-9
    field = philox.initial_field(seed, 0, 0, L).astype(np.int64)
    for code in out["flips"][0]:
        field[code % L] *= -1
    Gu, Gd = OH.green_from_field(OH.g0_matrix(g0), field, OH.hs_lambda(U, beta / L))
    assert np.abs(out["green"][0, 0] - Gu).max() < 1e-8
    assert np.abs(out["green"][0, 1] - Gd).max() < 1e-8


def test_direct_recompute_beyond_its_lds_bound_is_refused(ctx):
    import paper_0801_1222_amd as P
    beta, L = 160.0, 3200
    g0 = OB.bath_to_tau(OB.semicircle_iw(beta, 1.0, 4000), 1.0, beta, L)
    with pytest.raises(P.HFQMCError) as e:
        P.hfqmc_solve(ctx, g0, 4.0, beta, beta / L, 1, n_chains=1, warmup=0, sweeps=1,
                      mode="delayed", delay_k=32, n_bins=1, direct=True)
    assert e.value.code == -6 and "LDS" in str(e.value)
