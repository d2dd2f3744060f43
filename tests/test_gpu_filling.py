"""GPU tests away from half filling (the two-matrix path takes any bath).

The Hubbard atom on a level eps0 (chemical potential -eps0) is Trotter-exact
for every L, with a closed form for G(tau) and D: the Monte Carlo result must
agree within its error bars.  With the same (particle-hole asymmetric) bath,
the GPU chains must take the oracle's flips and match its accumulators within
1e-10 (FP64 paths).
"""
import numpy as np
import pytest

from oracle import hfqmc as OH

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch  # noqa: F401  (PyTorch's runtime comes up before the library's)
    import paper_0801_1222_amd as P
    c = P.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("mode,k", [("rank1", 0), ("delayed", 16)])
def test_asymmetric_bath_matches_oracle(ctx, mode, k):
    import paper_0801_1222_amd as P
    beta, U, L, eps0, seed = 6.0, 3.0, 30, -0.6, 2
    g0 = OH.atomic_level_bath(eps0, beta, np.arange(L) * beta / L)
    n_rec = 100 if mode == "rank1" else 4 * k
    out = P.hfqmc_solve(ctx, g0, U, beta, beta / L, seed, n_chains=3, warmup=3, sweeps=20,
                        mode=mode, delay_k=k, flip_cap=20000, want_chain=True)
    for c in range(3):
        ref = OH.run_chain(g0, U, beta, seed, chain=c, warmup=3, sweeps=20, n_rec=n_rec)
        assert list(out["flips"][c]) == [sw * L + l for sw, l in ref["flips"]]
        n = out["chain_n"][c][0]
        assert np.abs(out["chain_g"][c][0] / n - ref["bins_g"][0] / ref["bins_n"][0]).max() < 1e-10
        assert abs(out["chain_d"][c][0] / n - ref["bins_d"][0] / ref["bins_n"][0]) < 1e-10


@pytest.mark.parametrize("eps0,mode", [(-0.7, "delayed"), (0.5, "mixed"), (-1.2, "rank1")])
def test_atomic_level_monte_carlo_matches_closed_form(ctx, eps0, mode):
    import paper_0801_1222_amd as P
    beta, U, L = 4.0, 4.0, 16
    tau = np.arange(L) * beta / L
    g0 = OH.atomic_level_bath(eps0, beta, tau)
    out = P.hfqmc_solve(ctx, g0, U, beta, beta / L, 13, n_chains=64, warmup=20, sweeps=400,
                        mode=mode, delay_k=16 if mode != "rank1" else 0)
    exact = OH.atomic_level_g(eps0, U, beta, np.arange(L + 1) * beta / L)
    z = np.abs(out["g"] - exact)[1:L] / out["g_err"][1:L]
    assert z.max() < 4.5
    # G(0+) = 1 - n and G(beta-) = n hold exactly for every sample
    assert abs(out["g"][0] + out["g"][L] - 1.0) < 1e-12
    assert abs(out["D"] - OH.atomic_level_d(eps0, U, beta)) < 4.5 * out["D_err"]
