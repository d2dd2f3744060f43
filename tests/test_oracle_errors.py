"""Pins of the oracle's error bars and of the Neel cycle's crossed closure.

Every statistical gate of the GPU tests (3 sigma of the combined error) rests
on these error bars, and the GPU's chain reduction is matched to the oracle's
at 1e-9, so a wrong formula on both sides would make those gates vacuous.
Pinned here against things other than the oracle's own formulas:

  * chain and bin error bars (reading: standard error over chains, or over
    bins of a single chain): independent solves of the semicircle bath at
    beta = 10, U = 4, L = 12 scatter around the exact enumeration value with
    chi^2 per point near 1, and the spread of their estimates over the seeds
    matches the error bars they report;
  * the extrapolation's error (section "Multigrid HF-QMC method", step (ii)):
    the standard deviation of c0 over Gaussian-noised polynomial data equals
    the reported error within the Monte Carlo accuracy;
  * the Neel cycle's crossed closure: at U = 0 every grid returns its bath,
    so one iteration with unequal baths must close spin up over the spin-down
    bath and vice versa, exactly.
"""
import os

import numpy as np
import pytest

from oracle import bath as B
from oracle import hfqmc as H
from oracle import multigrid as MG

HERE = os.path.dirname(os.path.abspath(__file__))


def _exact_l12():
    g = {}
    D = None
    with open(os.path.join(HERE, "golden", "bethe_b10_u4_L12.txt")) as f:
        for line in f:
            if line.startswith("D "):
                D = float(line.split()[1])
            elif line.startswith("G "):
                k, v = line.split()[1:]
                g[int(k)] = float(v)
    return np.array([g[k] for k in range(len(g))]), D


def _calibration(results, g_exact, d_exact, L):
    """chi^2 per point against the exact values (D and G(tau_k), 0 < k < L) and the
    ratio of the spread of the estimates over seeds to the rms reported error."""
    g = np.array([r[0][1:L] for r in results])
    ge = np.array([r[1][1:L] for r in results])
    d = np.array([r[2] for r in results])
    de = np.array([r[3] for r in results])
    z = np.concatenate([((g - g_exact[1:L]) / ge).ravel(), (d - d_exact) / de])
    chi2 = float(np.mean(z * z))
    spread_g = np.std(g, axis=0, ddof=1) / np.sqrt(np.mean(ge * ge, axis=0))
    spread_d = np.std(d, ddof=1) / np.sqrt(np.mean(de * de))
    return chi2, float(np.mean(spread_g)), float(spread_d)


@pytest.mark.parametrize("n_chains,sweeps,n_bins", [(16, 160, 1), (1, 1600, 16)])
def test_error_bars_match_the_scatter_of_independent_solves(n_chains, sweeps, n_bins):
    # 24 independent solves (disjoint seeds); chains averaged (standard error over
    # chains) or one chain binned (standard error over bins)
    beta, U, L = 10.0, 4.0, 12
    g_tau = B.bath_to_tau(B.semicircle_iw(beta, 1.0, 20000), 1.0, beta, L)
    g_exact, d_exact = _exact_l12()
    res = []
    for s in range(24):
        r = H.solve(g_tau, U, beta, seed=(s + 1) * 1000003, n_chains=n_chains, warmup=40,
                    sweeps=sweeps, n_bins=n_bins)
        res.append((r["g"], r["g_err"], r["D"], r["D_err"]))
    chi2, spread_g, spread_d = _calibration(res, g_exact, d_exact, L)
    # t statistics with n - 1 = 15 degrees of freedom have E[t^2] = 15/13
    assert 0.6 < chi2 < 1.6, chi2
    # the standard deviation of 24 estimates is known to about 15 %
    assert 0.7 < spread_g < 1.35, spread_g
    assert 0.6 < spread_d < 1.45, spread_d


def test_extrapolation_error_is_the_scatter_of_c0():
    # Gaussian noise of known, unequal sigma on data exactly quadratic in dtau^2:
    # the reported error of c0 must be the standard deviation of c0 itself
    dts = np.array([0.4, 1 / 3, 2 / 7, 0.25, 0.2])
    f0, a, b = 0.083, -0.21, 0.9
    truth = f0 + a * dts ** 2 + b * dts ** 4
    sig = np.array([3e-4, 2e-4, 1.5e-4, 1.2e-4, 2.5e-4])
    rng = np.random.default_rng(2024)
    n = 4000
    gi = truth[:, None] + sig[:, None] * rng.standard_normal((dts.size, n))
    c0, err = MG.extrapolate(dts, gi, np.repeat(sig[:, None], n, axis=1))
    assert np.allclose(err, err[0], rtol=0, atol=0)     # depends on sigma only
    sd = np.std(c0, ddof=1)
    assert abs(sd / err[0] - 1.0) < 0.15, (sd, err[0])
    assert abs(np.mean(c0) - f0) < 4.0 * err[0] / np.sqrt(n)


def test_neel_cycle_closes_each_spin_over_the_other():
    # U = 0 and unequal baths of the same 1/(i w)^3 moment t^2: every grid returns
    # its spin's bath exactly, so the new baths must be the Bethe closures of the
    # OTHER spin's bath
    beta, t = 10.0, 1.0
    b_up = B.semicircle_iw(beta, t, 2000)
    b_dn = B.atomic_seed_iw(beta, t, 3.0, 2000)
    assert np.abs(b_up - b_dn).max() > 0.1
    r = MG.dmft_loop_af((b_up, b_dn), 0.0, beta, t, [0.5, 0.4, 0.25], 1, 1, n_chains=2,
                        warmup=1, sweeps=2, n_fine=101)
    new_up, new_dn = r["baths"]
    assert np.abs(new_up - B.bethe_step_iw(b_dn, beta, t)).max() < 1e-10
    assert np.abs(new_dn - B.bethe_step_iw(b_up, beta, t)).max() < 1e-10
    # and the returned G of each spin is its own bath (not the other's)
    tau = r["tau"]
    for sp, b in ((0, b_up), (1, b_dn)):
        exact = B.iw_to_tau(b, t * t, beta, tau)
        exact[-1] = 1.0 - exact[0]
        assert np.abs(r["g"][sp] - exact).max() < 1e-10
