"""Pins of the oracle away from half filling (the method's generality, closing remarks).

  * The 1/(i w)^2 moment of the Matsubara -> tau transform: the bath of a bare
    level eps, 1/(i w - eps) (moments eps, eps^2), against its closed form
    e^{-eps tau}/(1 + e^{-beta eps}); the Bethe lattice at chemical potential
    mu against the independent real-frequency quadrature in tau.
  * The lattice Green function at mu against the same quadrature on the
    Matsubara axis, and as the U = 0 fixed point of the cycle at mu.
  * The reference model at n = 1/2 is the half-filled one.
  * The multigrid step at any filling on the Hubbard atom on a level
    (Trotter-exact on every grid): the extrapolated G(tau) and D within their
    errors of the closed form.
"""
import numpy as np
import pytest

from oracle import bath as B
from oracle import hfqmc as H
from oracle import multigrid as MG


@pytest.mark.parametrize("eps,beta", [(0.7, 10.0), (-1.3, 5.0), (0.2, 40.0)])
def test_level_bath_transform_has_the_second_moment(eps, beta):
    n_iw = 20000
    iw = 1j * B.matsubara(beta, n_iw)
    tau = np.linspace(0.0, beta, 41)[:-1]
    g = B.iw_to_tau(1.0 / (iw - eps), eps * eps, beta, tau, m2=eps)
    assert np.abs(g - H.atomic_level_bath(eps, beta, tau)).max() < 1e-11
    # without the moment the 1/(i w)^2 term stays in the sum, which converges
    # slowly at tau = 0+: an error of order |eps| beta / n_iw there
    g0 = B.iw_to_tau(1.0 / (iw - eps), eps * eps, beta, tau)
    assert np.abs(g0 - H.atomic_level_bath(eps, beta, tau))[0] > 1e-6


@pytest.mark.parametrize("mu", [0.5, -0.8, 1.5])
def test_lattice_green_function_at_mu(mu):
    beta, t = 10.0, 1.0
    g = B.bethe_lattice_iw(beta, t, mu, 4000)
    assert np.abs(g[:500] - B.bethe_lattice_iw_dos(beta, t, mu, 500)).max() < 1e-8
    assert np.all(g.imag < 0)
    # the closure at mu maps it onto itself (the U = 0 lattice solution)
    assert np.abs(B.bethe_step_iw(g, beta, t, mu=mu) - g).max() < 1e-12
    # its tail moments -mu, mu^2 + t^2 in the transform, against the tau quadrature
    tau = np.linspace(0.0, beta, 31)[:-1]
    gt = B.iw_to_tau(g, mu * mu + t * t, beta, tau, m2=-mu)
    assert np.abs(gt - B.semicircle_tau_dos(beta, t, tau, mu=mu)).max() < 1e-7


def test_reference_at_half_density_is_the_half_filled_one():
    beta, U = 10.0, 3.0
    bath = B.semicircle_iw(beta, 1.0, 2000)
    assert np.abs(MG.reference_iw_n(bath, U, beta, 0.5) - MG.reference_iw(bath, U, beta)).max() < 1e-15
    M2, M3 = MG.reference_moments(0.0, 1.0, U, 0.5)
    assert M2 == 0.0 and abs(M3 - (1.0 + 0.25 * U * U)) < 1e-15


def test_reference_tail_moments_match_its_transform():
    # G_ref's transform with the moments of reference_moments is continuous across
    # the frequency cut: a wrong moment shows as a mismatch between two cut-offs
    beta, U, mu, t, n = 8.0, 2.5, 0.6, 1.0, 0.63
    bath = B.bethe_lattice_iw(beta, t, mu, 16000)
    tau = np.linspace(0.0, beta, 17)[:-1]
    a = MG.reference_tau_n(bath[:4000], -mu, mu * mu + t * t, U, beta, tau, n)
    b = MG.reference_tau_n(bath, -mu, mu * mu + t * t, U, beta, tau, n)
    assert np.abs(a - b).max() < 1e-9


def test_u0_cycle_at_mu_is_a_fixed_point():
    beta, t, mu = 10.0, 1.0, 0.6
    bath = B.bethe_lattice_iw(beta, t, mu, 4000)
    r = MG.dmft_loop_mu(bath, 0.0, mu, beta, t, [0.5, 0.4, 0.25], 1, 2, n_chains=2, warmup=1,
                        sweeps=2, n_fine=81)
    assert r["history"][0][0] < 1e-10
    assert np.abs(r["bath"] - bath).max() < 1e-10
    # the density of the lattice at mu > 0 exceeds 1/2
    n = r["history"][-1][4]
    tau = np.array([0.0])
    assert abs(n - (1.0 - B.semicircle_tau_dos(beta, t, tau, mu=mu)[0])) < 1e-9
    assert n > 0.6


def test_atom_on_a_level_through_the_multigrid_step():
    # a bare level eps0 as bath: every grid is Trotter-exact for the Hubbard atom
    beta, U, eps0 = 4.0, 2.0, -0.6
    n_iw = 8000
    iw = 1j * B.matsubara(beta, n_iw)
    bath = 1.0 / (iw - eps0)
    out = MG.multigrid_solve_n(bath, eps0, eps0 * eps0, U, beta, [0.5, 0.4, 0.25], 7, 8, 30, 400,
                               n_fine=41)
    exact = H.atomic_level_g(eps0, U, beta, out["tau"])
    z = np.abs(out["g"] - exact)[1:-1] / out["g_err"][1:-1]
    assert z.max() < 4.0, z.max()
    assert abs(out["D"] - H.atomic_level_d(eps0, U, beta)) < 4.0 * out["D_err"]
    # G(beta-) = n is the finest grid's density, above 1/2 for eps0 < 0
    assert out["n_ref"] > 0.5
