"""Pins for the oracle's multigrid steps (interpolation, dtau^2 extrapolation).

* Data that is exactly quadratic in dtau^2 must extrapolate to its constant.
* U = 0: every HF-QMC grid returns the bath exactly, the reference model is
  the bath, so the end-to-end result is the bath on the fine grid.
* Hubbard atom: every grid is Trotter-exact, so the extrapolation must agree
  with the closed form within its error bar.
"""
import numpy as np

from oracle import bath as B
from oracle import hfqmc as H
from oracle import multigrid as MG


def test_extrapolation_exact_for_quadratic_in_dtau2():
    dts = [0.4, 0.333, 0.286, 0.25, 0.2]
    f = np.linspace(-0.3, 0.7, 9)
    a, b = 0.37, -1.3
    gi = np.array([f + a * d ** 2 + b * d ** 4 for d in dts])
    rng = np.random.default_rng(0)
    ei = rng.uniform(1e-4, 1e-3, size=gi.shape)
    c0, err = MG.extrapolate(dts, gi, ei)
    assert np.abs(c0 - f).max() < 1e-12
    assert np.all(err > 0)


def test_three_grids_fit_is_exact_interpolation():
    dts = [0.125, 0.1, 0.0625]
    rng = np.random.default_rng(1)
    gi = rng.normal(size=(3, 7))
    c0, _ = MG.extrapolate(dts, gi, np.full(gi.shape, 1e-3))
    x = np.array(dts) ** 2
    for j in range(7):
        coef = np.polyfit(x, gi[:, j], 2)
        assert abs(coef[-1] - c0[j]) < 1e-9


def test_interpolation_returns_reference_when_data_is_reference():
    beta = 10.0
    bath = B.semicircle_iw(beta, 1.0, 2000)
    L = 40
    tau_k = np.arange(L + 1) * beta / L
    tf = MG.fine_grid(beta, 200)
    gk = MG.reference_tau(bath, 1.0, 3.0, beta, tau_k)
    gf_ref = MG.reference_tau(bath, 1.0, 3.0, beta, tf)
    gf, _ = MG.interpolate_grid(gk, np.zeros(L + 1), beta, gk, gf_ref, tf)
    assert np.abs(gf - gf_ref).max() == 0.0


def test_u0_multigrid_is_exact():
    beta = 10.0
    bath = B.semicircle_iw(beta, 1.0, 4000)
    out = MG.multigrid_solve(bath, 1.0, 0.0, beta, [0.5, 0.4, 0.25], seed=0,
                             n_chains=2, warmup=1, sweeps=2, n_fine=60)
    exact = B.iw_to_tau(bath, 1.0, beta, out["tau"])
    # tau = beta- is the left limit: G(beta-) = 1 - G(0+)
    exact[-1] = 1.0 - exact[0]
    assert np.abs(out["g"] - exact).max() < 1e-12


def test_atomic_limit_multigrid_within_errors():
    beta, U = 4.0, 4.0
    bath = 1.0 / (1j * B.matsubara(beta, 4000))
    out = MG.multigrid_solve(bath, 0.0, U, beta, [0.5, 0.4, 0.25], seed=5,
                             n_chains=4, warmup=30, sweeps=400, n_fine=41)
    exact = H.atomic_limit_g(U, beta, out["tau"])
    z = np.abs(out["g"] - exact)[1:-1] / out["g_err"][1:-1]
    assert z.max() < 4.0
    # the extrapolated double occupancy as well (every grid is Trotter-exact)
    assert abs(out["D"] - H.atomic_limit_d(U, beta)) < 4.0 * out["D_err"]


def test_u0_double_occupancy_is_a_quarter():
    # U = 0: D = <n_up><n_dn> = 1/4 exactly on every grid and after the fit
    beta = 10.0
    bath = B.semicircle_iw(beta, 1.0, 4000)
    out = MG.multigrid_solve(bath, 1.0, 0.0, beta, [0.5, 0.4, 0.25], seed=0,
                             n_chains=2, warmup=1, sweeps=2, n_fine=60)
    assert abs(out["D"] - 0.25) < 1e-12


def test_dmft_loop_u0_semicircle_is_fixed_point():
    # U = 0: every grid returns the bath exactly, the extrapolation and the
    # reference model are exact, and the semicircle solves the Bethe closure
    beta, t = 10.0, 1.0
    bath = B.semicircle_iw(beta, t, 4000)
    out = MG.dmft_loop(bath, 0.0, beta, t, [0.5, 0.4, 0.25], seed=1, n_iter=2, n_chains=2,
                       warmup=1, sweeps=2, n_fine=200)
    assert out["history"][0][0] < 1e-12           # G(tau) is the bath's own G0(tau)
    assert np.abs(out["bath"] - bath).max() < 1e-10
    # the second iteration starts from that bath: still self-consistent
    assert out["history"][1][0] < 1e-10


def test_dmft_loop_keeps_particle_hole_symmetry():
    # the estimator averages both spins, so G(tau) = G(beta - tau) for every
    # sample; the closure of a symmetric G is a purely imaginary bath
    beta, U, t = 4.0, 4.0, 1.0
    bath = B.semicircle_iw(beta, t, 2000)
    out = MG.dmft_loop(bath, U, beta, t, [0.5, 0.4, 0.25], seed=3, n_iter=1, n_chains=2,
                       warmup=5, sweeps=40, n_fine=81)
    g = out["g"]
    assert np.abs(g - g[::-1]).max() < 1e-10
    assert np.abs(out["bath"].real).max() < 1e-10
    assert np.all(out["bath"].imag < 0)
    # an interacting bath moved away from the semicircle
    assert np.abs(out["bath"] - bath).max() > 1e-3


def test_af_cycle_u0_semicircle_is_fixed_point():
    # U = 0: each spin's G is its bath, and the crossed closure returns the semicircle
    beta, t = 10.0, 1.0
    b = B.semicircle_iw(beta, t, 2000)
    r = MG.dmft_loop_af((b, b), 0.0, beta, t, [0.5, 0.4, 0.25], 1, 2, n_chains=2, warmup=1,
                        sweeps=3, n_fine=81)
    assert np.abs(r["baths"][0] - b).max() < 1e-12 and np.abs(r["baths"][1] - b).max() < 1e-12
    assert np.abs(r["history"][:, 4]).max() < 1e-13


def test_spin_multigrid_with_equal_baths_averages_to_plain_multigrid():
    # the same chains: per grid, the mean of the two spins' interpolated G equals
    # the spin-averaged solve's (extrapolations differ only through their weights)
    beta, U, t = 4.0, 3.0, 1.0
    b = B.semicircle_iw(beta, t, 2000)
    kw = dict(n_chains=2, warmup=2, sweeps=10, n_fine=41)
    a = MG.multigrid_solve(b, t * t, U, beta, [0.5, 0.4, 0.25], 5, **kw)
    s = MG.multigrid_solve_spin((b, b), t * t, U, beta, [0.5, 0.4, 0.25], 5, **kw)
    assert np.abs(s["g_interp"].mean(axis=1) - a["g_interp"]).max() < 1e-12
    assert abs(s["D"] - a["D"]) < 1e-12
