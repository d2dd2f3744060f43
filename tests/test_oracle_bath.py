"""Pins for the oracle's bath and Fourier routines.

* Matsubara route vs an independent real-frequency quadrature of the
  semicircular density of states (Benchmark section: W = 4, t = 1).
* Particle-hole symmetry G(tau) = G(beta - tau) and G(0+) = 1/2.
* The semicircle is a fixed point of the Bethe closure at U = 0.
* The reference model reduces to the closed-form Hubbard atom.
* Spline Fourier integral converges to a closed-form G(i w).
* The insulating seed (Bethe closure of the Hubbard atom) against its
  imaginary-time closed form from a partial-fraction expansion.
"""
import numpy as np
import pytest

from oracle import bath as B
from oracle import hfqmc as H
from oracle import multigrid as MG


@pytest.mark.parametrize("beta,L", [(10.0, 20), (40.0, 400), (20.0, 160)])
def test_matsubara_route_matches_dos_quadrature(beta, L):
    g_iw = B.semicircle_iw(beta, 1.0, 20000)
    g = B.bath_to_tau(g_iw, 1.0, beta, L)
    tau = np.arange(L) * beta / L
    sel = np.unique(np.linspace(0, L - 1, 25).astype(int))
    ref = B.semicircle_tau_dos(beta, 1.0, tau[sel], n_nodes=40000)
    assert np.abs(g[sel] - ref).max() < 5e-11


def test_half_filling_symmetries():
    beta, L = 10.0, 20
    g = B.bath_to_tau(B.semicircle_iw(beta, 1.0, 20000), 1.0, beta, L)
    assert abs(g[0] - 0.5) < 1e-14
    # G(tau_k) = G(beta - tau_k) = G(tau_{L-k})
    assert np.abs(g[1:] - g[1:][::-1]).max() < 1e-13
    assert np.all(np.diff(g[: L // 2 + 1]) < 0)


def test_semicircle_is_bethe_fixed_point_at_u0():
    beta, t = 10.0, 1.0
    b0 = B.semicircle_iw(beta, t, 4000)
    tf = MG.fine_grid(beta, 200)
    gf = B.iw_to_tau(b0, t * t, beta, tf)
    nb = MG.dmft_bethe_step(gf, tf, b0, t * t, 0.0, beta, t)
    assert np.abs(nb - b0).max() < 1e-12


def test_reference_model_atomic_limit():
    beta, U = 10.0, 4.0
    b_at = 1.0 / (1j * B.matsubara(beta, 4000))
    tau = np.linspace(0.0, beta, 21)
    ref = MG.reference_tau(b_at, 0.0, U, beta, tau)
    assert np.abs(ref - H.atomic_limit_g(U, beta, tau)).max() < 1e-12


def test_spline_fourier_converges_to_closed_form():
    # True G = semicircle; the reference model (U = 1) differs from it, so
    # the spline carries a nonzero smooth difference that must transform back.
    beta = 10.0
    b0 = B.semicircle_iw(beta, 1.0, 2000)
    errs = []
    for nf in (100, 200, 400):
        tf = MG.fine_grid(beta, nf)
        gf = B.iw_to_tau(b0, 1.0, beta, tf)
        giw = MG.g_tau_to_iw(gf, tf, b0, 1.0, 1.0, beta)
        errs.append(np.abs(giw - b0).max())
    assert errs[-1] < 2e-7
    assert errs[0] / errs[1] > 6 and errs[1] / errs[2] > 6


@pytest.mark.parametrize("beta,U,L", [(45.0, 5.0, 90), (10.0, 0.0, 40), (20.0, 3.0, 57)])
def test_atomic_seed_matches_partial_fractions(beta, U, L):
    # 1/(z - t^2 z/(z^2 - a)) = (z^2 - a)/(z (z^2 - E^2)), a = U^2/4, E^2 = a + t^2:
    # poles 0 (weight a/E^2) and +-E (weight t^2/(2 E^2) each); a pole at e
    # contributes w e^{-tau e}/(1 + e^{-beta e}) to the positive-convention G(tau)
    t = 1.0
    b = B.atomic_seed_iw(beta, t, U, 20000)
    g = B.bath_to_tau(b, t * t, beta, L)
    tau = np.arange(L) * beta / L
    a = U * U / 4.0
    E = np.sqrt(a + t * t)
    exact = (a / E ** 2) / 2.0 + t * t / (2.0 * E * E) * (
        np.exp(-tau * E) + np.exp(-(beta - tau) * E)) / (1.0 + np.exp(-beta * E))
    assert np.abs(g - exact).max() < 1e-12
    # high-frequency moment t^2 (the same tail as the semicircle)
    w = B.matsubara(beta, 20000)[-1]
    assert abs((b[-1] - 1.0 / (1j * w)) * (1j * w) ** 3 - t * t) < 1e-6
