"""GPU parity of the multigrid DMFT cycle away from half filling (through the C ABI).

The method's generality (closing remarks): at chemical potential mu the bath
carries a 1/(i w)^2 moment, the Bethe closure reads 1/(i w + mu - t^2 G), and
the reference model of the interpolation is taken at the density n.  Checked
against the oracle's cycle (identical chains in FP64: 1e-9 on G, its errors,
the new bath and the history), the U = 0 lattice at mu as a fixed point, and
the Hubbard atom on a level through the multigrid step against its closed form.
"""
import numpy as np
import pytest

from oracle import bath as OB
from oracle import hfqmc as OH
from oracle import multigrid as OMG

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch  # noqa: F401  (PyTorch's runtime comes up before the library's)
    import paper_0801_1222_amd as P
    c = P.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("mode,k", [("rank1", 0), ("delayed", 16)])
def test_dmft_cycle_at_mu_matches_oracle(ctx, mode, k):
    import paper_0801_1222_amd as P
    beta, U, mu, t = 4.0, 2.5, 0.7, 1.0
    dtaus = [0.5, 0.4, 0.25]
    n_iw, n_fine, seed = 2048, 81, 11
    kw = dict(n_chains=4, warmup=5, sweeps=30, mode=mode, delay_k=k, recompute_every=40)
    bath = OB.bethe_lattice_iw(beta, t, mu, n_iw)
    ref = OMG.dmft_loop_mu(bath, U, mu, beta, t, dtaus, seed, 2, 4, 5, 30, n_rec=40,
                           n_fine=n_fine, mixing=0.3)
    out = P.dmft_solve_mu(ctx, U, mu, beta, t, dtaus, seed, 2, bath_iw=bath, n_fine=n_fine,
                          mixing=0.3, **kw)
    assert np.abs(out["g"] - ref["g"]).max() < 1e-9
    assert np.abs(out["g_err"] - ref["g_err"]).max() < 1e-9
    assert np.abs(out["bath"] - ref["bath"]).max() < 1e-9
    assert np.abs(out["history"] - ref["history"]).max() < 1e-9
    # away from half filling: n > 1/2 for mu > 0, and G(tau) is not symmetric
    assert out["history"][-1][4] > 0.55
    assert np.abs(out["g"] - out["g"][::-1]).max() > 1e-2


def test_u0_lattice_at_mu_is_a_fixed_point(ctx):
    import paper_0801_1222_amd as P
    beta, mu, t = 10.0, -0.8, 1.0
    bath = P.bethe_lattice_bath(beta, t, mu, 4096)
    out = P.dmft_solve_mu(ctx, 0.0, mu, beta, t, [0.5, 0.4, 0.25], 3, 2, bath_iw=bath,
                          n_fine=101, n_chains=2, warmup=1, sweeps=2)
    assert out["history"][0][0] < 1e-10
    assert np.abs(out["bath"] - bath).max() < 1e-10
    assert out["history"][-1][4] < 0.35


def test_atom_on_a_level_through_the_multigrid_step(ctx):
    # a bare level eps0 as bath (tail moments eps0, eps0^2): Trotter-exact on every grid
    import paper_0801_1222_amd as P
    beta, U, eps0 = 4.0, 2.0, -0.6
    n_iw = 8192
    iw = 1j * OB.matsubara(beta, n_iw)
    bath = 1.0 / (iw - eps0)
    out = P.multigrid_solve_n(ctx, bath, eps0, eps0 * eps0, U, beta, [0.5, 0.4, 0.25], 7,
                              n_fine=41, n_chains=64, warmup=30, sweeps=400, mode="mixed",
                              delay_k=8)
    exact = OH.atomic_level_g(eps0, U, beta, out["tau"])
    z = np.abs(out["g"] - exact)[1:-1] / out["g_err"][1:-1]
    assert z.max() < 4.0, z.max()
    assert abs(out["D"] - OH.atomic_level_d(eps0, U, beta)) < 4.0 * out["D_err"]
    assert out["n_ref"] > 0.5
