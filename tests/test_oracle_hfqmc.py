"""Pins for the oracle's fixed-dtau Hirsch-Fye solver.

Each check is tied to something other than the oracle itself:
  * U = 0: lambda = 0, every update vanishes, G must equal the bath matrix and
    the estimator must return the bath G(tau_k) (closed form).
  * Hubbard atom (bath G(tau) = 1/2): the Trotter decomposition is exact, so
    the enumeration over all 2^L fields must give the closed-form atomic G(tau)
    and D for every L.
  * Determinant ratio and rank-1 update vs determinants and solves computed by
    LAPACK from scratch.
  * Particle-hole symmetry at half filling: G_dn = 1 - G_up^T per field.
  * Monte Carlo vs exact enumeration within statistical error (L <= 12).
  * Delayed updates reproduce the rank-1 sequence.
  * Spin-dependent baths (an atom in a Zeeman field): enumeration equals the
    closed form per spin; U = 0 returns each spin's own bath; one bath given
    twice reproduces the single-bath chain.
"""
import numpy as np
import pytest

from oracle import bath as B
from oracle import hfqmc as H
from oracle import philox


def _semicircle_tau(beta, L):
    return B.bath_to_tau(B.semicircle_iw(beta, 1.0, 20000), 1.0, beta, L)


def test_lambda_definition():
    for U, dt in [(4.0, 0.5), (4.5, 0.1), (5.0, 0.05)]:
        lam = H.hs_lambda(U, dt)
        assert abs(np.cosh(lam) - np.exp(0.5 * dt * U)) < 1e-13
    assert H.hs_lambda(0.0, 0.3) == 0.0


def test_u0_green_equals_bath():
    beta, L = 10.0, 16
    g = _semicircle_tau(beta, L)
    r = H.run_chain(g, 0.0, beta, seed=3, warmup=1, sweeps=4)
    G0 = H.g0_matrix(g)
    assert np.abs(r["Gu"] - G0).max() == 0.0
    assert np.abs(r["Gd"] - G0).max() == 0.0
    est = r["bins_g"][0] / r["bins_n"][0]
    assert np.abs(est[:L] - g).max() < 1e-15
    assert abs(est[L] - (1.0 - g[0])) < 1e-15
    assert r["n_accepted"] == r["n_proposed"]


def test_bath_matrix_is_antiperiodic():
    g = np.arange(1, 7, dtype=float)
    G0 = H.g0_matrix(g)
    L = g.size
    for i in range(L):
        for j in range(L):
            k = i - j
            assert G0[i, j] == (g[k] if k >= 0 else -g[k + L])


@pytest.mark.parametrize("beta,U,L", [(4.0, 4.0, 6), (10.0, 4.0, 10), (3.0, 6.0, 8)])
def test_atomic_limit_enumeration_is_exact(beta, U, L):
    g = np.full(L, 0.5)
    gb, Db, wmin = H.brute_force(g, U, beta)
    tau = np.arange(L + 1) * beta / L
    assert wmin > 0.0
    assert np.abs(gb - H.atomic_limit_g(U, beta, tau)).max() < 1e-13
    assert abs(Db - H.atomic_limit_d(U, beta)) < 1e-14


def test_atomic_limit_monte_carlo():
    beta, U, L = 4.0, 4.0, 10
    res = H.solve(np.full(L, 0.5), U, beta, seed=11, n_chains=4, warmup=50, sweeps=1500)
    tau = np.arange(L + 1) * beta / L
    z = np.abs(res["g"] - H.atomic_limit_g(U, beta, tau)) / np.maximum(res["g_err"], 1e-12)
    assert z[1:L].max() < 4.0
    assert abs(res["D"] - H.atomic_limit_d(U, beta)) < 4.0 * res["D_err"]


def test_flip_ratio_is_determinant_ratio():
    beta, U, L = 10.0, 4.0, 12
    g = _semicircle_tau(beta, L)
    lam = H.hs_lambda(U, beta / L)
    gp, gm = H.flip_gammas(lam)
    G0 = H.g0_matrix(g)
    s = philox.initial_field(5, 0, 0, L).astype(np.int64)
    Gu, Gd = H.green_from_field(G0, s, lam)
    for l in range(L):
        s2 = s.copy()
        s2[l] = -s2[l]
        _, _, ru, rd, R = H.flip_ratio(Gu[l, l], Gd[l, l], s[l], gp, gm)
        du = np.linalg.det(H.dyson_matrix(G0, s2, lam, 1)) / np.linalg.det(H.dyson_matrix(G0, s, lam, 1))
        dd = np.linalg.det(H.dyson_matrix(G0, s2, lam, -1)) / np.linalg.det(H.dyson_matrix(G0, s, lam, -1))
        assert abs(ru - du) < 1e-11 * abs(du)
        assert abs(rd - dd) < 1e-11 * abs(dd)
        assert R > 0


def test_rank1_update_equals_recompute():
    beta, U, L = 10.0, 4.0, 20
    g = _semicircle_tau(beta, L)
    lam = H.hs_lambda(U, beta / L)
    gp, gm = H.flip_gammas(lam)
    G0 = H.g0_matrix(g)
    s = philox.initial_field(1, 0, 0, L).astype(np.int64)
    Gu, Gd = H.green_from_field(G0, s, lam)
    rng = np.random.default_rng(0)
    for _ in range(100):
        l = int(rng.integers(L))
        gu, gd, ru, rd, _ = H.flip_ratio(Gu[l, l], Gd[l, l], s[l], gp, gm)
        H.rank1_update(Gu, l, gu / ru)
        H.rank1_update(Gd, l, gd / rd)
        s[l] = -s[l]
        nu, nd = H.green_from_field(G0, s, lam)
        assert max(np.abs(nu - Gu).max(), np.abs(nd - Gd).max()) < 1e-11


def test_particle_hole_identity_per_field():
    beta, U, L = 10.0, 4.0, 20
    g = _semicircle_tau(beta, L)
    lam = H.hs_lambda(U, beta / L)
    G0 = H.g0_matrix(g)
    for seed in range(5):
        s = philox.initial_field(seed, 0, 0, L).astype(np.int64)
        Gu, Gd = H.green_from_field(G0, s, lam)
        assert np.abs(Gd - (np.eye(L) - Gu.T)).max() < 1e-12
        est, _ = H.measure(Gu, Gd)
        # spin-averaged estimator is symmetric per configuration: G(tau_k) = G(tau_{L-k})
        assert np.abs(est[1:L] - est[1:L][::-1]).max() < 1e-13
        assert abs(est[0] - 0.5) < 1e-14


def test_enumeration_weights_positive_and_symmetric():
    beta, U, L = 4.0, 4.0, 8
    g = _semicircle_tau(beta, L)
    gb, Db, wmin = H.brute_force(g, U, beta)
    assert wmin > 0.0
    assert np.abs(gb[1:L] - gb[1:L][::-1]).max() < 1e-13
    assert abs(gb[0] - 0.5) < 1e-13 and abs(gb[L] - 0.5) < 1e-13
    assert 0.0 < Db < 0.25


def test_monte_carlo_matches_enumeration_L12():
    beta, U, L = 10.0, 4.0, 12
    g = _semicircle_tau(beta, L)
    gb, Db, _ = H.brute_force(g, U, beta)
    res = H.solve(g, U, beta, seed=0, n_chains=1, warmup=100, sweeps=4000)
    z = np.abs(res["g"][1:L] - gb[1:L]) / res["g_err"][1:L]
    assert z.max() < 3.5
    assert abs(res["D"] - Db) < 3.5 * res["D_err"]
    c = res["chains"][0]
    assert c["n_bad"] == 0
    assert c["max_drift"] < 1e-11
    assert c["n_recomputes"] == c["n_accepted"] // 100


def test_heat_bath_matches_enumeration_L12():
    # heat-bath acceptance samples the same distribution: same exact answer,
    # a lower acceptance rate than Metropolis on the same stream
    beta, U, L = 10.0, 4.0, 12
    g = _semicircle_tau(beta, L)
    gb, Db, _ = H.brute_force(g, U, beta)
    res = H.solve(g, U, beta, seed=0, n_chains=1, warmup=100, sweeps=4000, heat_bath=True)
    z = np.abs(res["g"][1:L] - gb[1:L]) / res["g_err"][1:L]
    assert z.max() < 3.5
    assert abs(res["D"] - Db) < 3.5 * res["D_err"]
    met = H.run_chain(g, U, beta, seed=0, warmup=0, sweeps=200)
    hb = H.run_chain(g, U, beta, seed=0, warmup=0, sweeps=200, heat_bath=True)
    assert hb["n_accepted"] < met["n_accepted"]


def test_delayed_updates_reproduce_rank1():
    beta, U, L = 10.0, 4.0, 20
    g = _semicircle_tau(beta, L)
    r1 = H.run_chain(g, U, beta, seed=3, warmup=2, sweeps=30, n_rec=100)
    for k in (1, 4, 7):
        r2 = H.run_chain(g, U, beta, seed=3, warmup=2, sweeps=30, n_rec=100, delay_k=k)
        assert r1["flips"] == r2["flips"]
        assert np.abs(r1["bins_g"] - r2["bins_g"]).max() < 1e-11
        assert np.abs(r1["Gu"] - r2["Gu"]).max() < 1e-12


def test_fp32_flush_drift_is_small_under_replay():
    beta, U, L = 10.0, 4.5, 50
    g = _semicircle_tau(beta, L)
    r1 = H.run_chain(g, U, beta, seed=2, warmup=0, sweeps=20, n_rec=64)
    rep = set(r1["flips"])
    r2 = H.run_chain(g, U, beta, seed=2, warmup=0, sweeps=20, n_rec=64, delay_k=16,
                     flush_fp32=True, replay=rep)
    assert r2["flips"] == r1["flips"]
    n = r1["bins_n"][0]
    assert np.abs(r1["bins_g"][0] - r2["bins_g"][0]).max() / n < 1e-5
    assert 0.0 < r2["max_drift"] < 1e-4


def test_replay_of_own_flips_is_identical():
    beta, U, L = 10.0, 4.0, 20
    g = _semicircle_tau(beta, L)
    r1 = H.run_chain(g, U, beta, seed=9, warmup=1, sweeps=10)
    r2 = H.run_chain(g, U, beta, seed=9, warmup=1, sweeps=10, replay=set(r1["flips"]))
    assert r1["flips"] == r2["flips"]
    assert np.array_equal(r1["bins_g"], r2["bins_g"])


def test_atomic_level_reduces_to_half_filled_atom():
    beta, U = 4.0, 3.0
    tau = np.linspace(0.0, beta, 9)
    assert np.abs(H.atomic_level_g(0.0, U, beta, tau) - H.atomic_limit_g(U, beta, tau)).max() < 1e-14
    assert abs(H.atomic_level_d(0.0, U, beta) - H.atomic_limit_d(U, beta)) < 1e-15
    assert np.abs(H.atomic_level_bath(0.0, beta, tau[:-1]) - 0.5).max() == 0.0
    # U = 0: the interacting atom is its own bath
    assert np.abs(H.atomic_level_g(-0.6, 0.0, beta, tau[:-1])
                  - H.atomic_level_bath(-0.6, beta, tau[:-1])).max() < 1e-14


@pytest.mark.parametrize("eps0,L", [(-0.7, 8), (0.45, 10)])
def test_brute_force_atomic_level_away_from_half_filling(eps0, L):
    # general filling: exact enumeration of the HS field equals the closed form
    beta, U = 4.0, 4.0
    tau = np.arange(L) * beta / L
    g_tau = H.atomic_level_bath(eps0, beta, tau)
    g, d, wmin = H.brute_force(g_tau, U, beta)
    exact = H.atomic_level_g(eps0, U, beta, np.arange(L + 1) * beta / L)
    exact[L] = 1.0 - exact[0]
    assert wmin > 0
    assert np.abs(g - exact).max() < 1e-11
    assert abs(d - H.atomic_level_d(eps0, U, beta)) < 1e-12


def test_atomic_field_reduces_to_atomic_level_and_swaps_spins():
    beta, U = 4.0, 3.0
    tau = np.linspace(0.0, beta, 9)
    gu, gd = H.atomic_field_g(-0.4, -0.4, U, beta, tau)
    assert np.abs(gu - H.atomic_level_g(-0.4, U, beta, tau)).max() < 1e-14
    assert np.abs(gd - gu).max() == 0.0
    assert abs(H.atomic_field_d(-0.4, -0.4, U, beta) - H.atomic_level_d(-0.4, U, beta)) < 1e-15
    a, b = H.atomic_field_g(0.3, -0.5, U, beta, tau)
    c, d = H.atomic_field_g(-0.5, 0.3, U, beta, tau)
    assert np.abs(a - d).max() < 1e-15 and np.abs(b - c).max() < 1e-15


@pytest.mark.parametrize("eu,ed,L", [(-0.7, 0.3, 8), (0.5, -0.2, 10)])
def test_brute_force_spin_dependent_baths_match_closed_form(eu, ed, L):
    beta, U = 4.0, 4.0
    tau = np.arange(L) * beta / L
    baths = (H.atomic_level_bath(eu, beta, tau), H.atomic_level_bath(ed, beta, tau))
    gs, d, wmin = H.brute_force(baths, U, beta, spins=True)
    ex = np.array(H.atomic_field_g(eu, ed, U, beta, np.arange(L + 1) * beta / L))
    ex[:, L] = 1.0 - ex[:, 0]
    assert wmin > 0
    assert np.abs(gs - ex).max() < 1e-11
    assert abs(d - H.atomic_field_d(eu, ed, U, beta)) < 1e-12


def test_spin_dependent_chain_u0_and_equal_baths():
    beta, L = 5.0, 10
    tau = np.arange(L) * beta / L
    bu, bd = H.atomic_level_bath(-0.6, beta, tau), B.bath_to_tau(B.semicircle_iw(beta, 1.0, 8000), 1.0, beta, L)
    r = H.run_chain((bu, bd), 0.0, beta, 3, warmup=1, sweeps=4)
    assert np.abs(r["Gu"] - H.g0_matrix(bu)).max() < 1e-14
    assert np.abs(r["Gd"] - H.g0_matrix(bd)).max() < 1e-14
    m = r["bins_gs"][0] / r["bins_n"][0]
    assert np.abs(m[0, :L] - bu).max() < 1e-14 and np.abs(m[1, :L] - bd).max() < 1e-14
    # one bath given for both spins: the same chain as the single-bath call
    r1 = H.run_chain(bd, 4.0, beta, 5, warmup=1, sweeps=6)
    r2 = H.run_chain((bd, bd), 4.0, beta, 5, warmup=1, sweeps=6)
    assert r1["flips"] == r2["flips"]
    assert np.array_equal(r1["bins_g"], r2["bins_g"])
    assert np.abs(r2["bins_gs"][0].mean(axis=0) - r2["bins_g"][0]).max() < 1e-13
