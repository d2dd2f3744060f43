"""GPU study of coexisting metallic and insulating DMFT solutions (Benchmark
results section, Fig. 3: double occupancy against dtau^2 in both phases at
T = 1/45; semi-elliptic density of states of width 4, t = 1).

The multigrid DMFT cycle (four Trotter grids, dtau = 0.40 .. 0.25) is started
once from the metallic U = 0 semicircle and once from the insulating bath (the
Bethe closure of the Hubbard atom), at U = 4.8 inside the coexistence region.
Checks, all statistical (the paper prints no values to compare with):

* the two seeds converge to distinct fixed points: the metal keeps spectral
  weight at the Fermi level (G(beta/2) well above zero), the insulator does not,
  and their double occupancies are separated by many error bars;
* at each converged bath the raw double occupancy on seven grids, from coarser
  (dtau = 0.6) to finer (dtau = 0.2) than those of the cycle, is a smooth
  function of dtau^2: a quadratic in dtau^2 fits every point within its error,
  D grows monotonically as dtau -> 0, the metallic curve lies above the
  insulating one on every grid, and the extrapolated D agrees with the cycle's.

The insulating cycle is damped (mixing 0.5): undamped, rare large estimator
samples in the gapped phase can throw the iteration out of the insulating basin
at these statistics.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

BETA, U, T = 45.0, 4.8, 1.0
LS_CYCLE = [113, 129, 150, 180]
LS_STUDY = [75, 90, 113, 129, 150, 180, 225]
KW = dict(n_chains=256, warmup=100, sweeps=1000, mode="delayed", delay_k=16, ph=True)


@pytest.fixture(scope="module")
def phases():
    import torch  # noqa: F401  (PyTorch's runtime comes up before the library's)
    import paper_0801_1222_amd as P
    ctx = P.Context(0)
    dtaus = [BETA / L for L in LS_CYCLE]
    out = {}
    for name, bath, mixing in (("metal", P.bethe_semicircle_bath(BETA, T, 4096), 0.3),
                               ("insulator", P.bethe_atomic_bath(BETA, T, U, 4096), 0.5)):
        r = P.dmft_solve(ctx, U, BETA, T, dtaus, 3, 9, bath_iw=bath, n_fine=181, mixing=mixing, **KW)
        h = r["history"]
        print("%-9s D per iteration %s" % (name, " ".join("%.4f" % d for d in h[:, 2])), flush=True)
        out[name] = r
    out["ctx"] = ctx
    yield out
    ctx.close()


def test_metal_and_insulator_coexist(phases):
    met, ins = phases["metal"], phases["insulator"]
    for r in (met, ins):
        h = r["history"]
        # converged to the statistical noise of one iteration
        assert h[-1][0] < 8 * h[-1][1]
        assert abs(h[-1][2] - h[-2][2]) < 5e-4 + 5 * np.hypot(h[-1][3], h[-2][3])
        assert np.abs(r["bath"].real).max() == 0.0
    mid = met["g"].shape[0] // 2
    assert met["g"][mid] > 0.01 > 5 * met["g_err"][mid]
    assert abs(ins["g"][mid]) < 2e-3
    d_met, e_met = met["history"][-1][2:4]
    d_ins, e_ins = ins["history"][-1][2:4]
    assert 0.0 < d_ins < d_met < 0.25
    assert d_met - d_ins > 20 * np.hypot(e_met, e_ins), (d_met, e_met, d_ins, e_ins)


def test_double_occupancy_is_smooth_in_dtau_squared(phases):
    import paper_0801_1222_amd as P
    x = np.array([(BETA / L) ** 2 for L in LS_STUDY])
    curves = {}
    for name in ("metal", "insulator"):
        cyc = phases[name]
        m = P.multigrid_solve(phases["ctx"], cyc["bath"], T * T, U, BETA, [BETA / L for L in LS_STUDY],
                              99, n_fine=181, n_chains=128, warmup=100, sweeps=2000,
                              mode="delayed", delay_k=16, ph=True)
        assert m["Ls"] == LS_STUDY
        d, e = m["D_grids"], m["D_err_grids"]
        for st in m["stats"]:
            assert st["n_bad_ratio"] == 0 and st["n_singular"] == 0
        X = np.stack([np.ones_like(x), x, x * x], 1)
        coef = np.linalg.lstsq(X / e[:, None], d / e, rcond=None)[0]
        resid = (d - X @ coef) / e
        print("%-9s D(dtau^2): %s  extrapolated %.5f(%.0e)  residuals/sigma %s" % (
            name, " ".join("%.5f" % v for v in d), m["D"], m["D_err"],
            " ".join("%.1f" % r for r in resid)), flush=True)
        assert np.abs(resid).max() < 6.0
        # D rises towards dtau -> 0, by much more than the errors
        assert np.all(np.diff(d) > 5 * np.hypot(e[1:], e[:-1]))
        assert m["D"] > d[-1]
        # the extrapolation from seven grids agrees with the cycle's own from four
        d_cyc, e_cyc = cyc["history"][-1][2:4]
        assert abs(m["D"] - d_cyc) < 5e-4 + 5 * np.hypot(m["D_err"], e_cyc)
        curves[name] = (d, e)
    (dm, em), (di, ei) = curves["metal"], curves["insulator"]
    assert np.all(dm - di > 10 * np.hypot(em, ei))
