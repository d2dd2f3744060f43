"""GPU tests of the Neel-order DMFT cycle (dmft_solve_af) on the Bethe lattice:
spin-dependent baths through the multigrid step, crossed closure
Bath_sigma = 1/(i w - t^2 G_-sigma).

* U = 0: the semicircle is a fixed point; no moment appears.
* Parity: the C-ABI cycle against the oracle's (same Philox streams per
  iteration, FP64 rank-1): identical arithmetic up to rounding.
* Physics at half filling, U = 3, T = 1/20 (well inside the antiferromagnetic
  phase of the half-filled Bethe lattice): from a weakly staggered start the
  moment grows to a large value, and the solution keeps the particle-hole
  symmetry of the Neel state, G_dn(tau) = G_up(beta - tau), within errors.
  Statistical only: the paper prints no magnetic data.
"""
import numpy as np
import pytest

from oracle import bath as OB
from oracle import multigrid as OM

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch  # noqa: F401  (PyTorch's runtime comes up before the library's)
    import paper_0801_1222_amd as P
    c = P.Context(0)
    yield c
    c.close()


def _staggered_baths(beta, t, h, n_iw):
    # G_sigma of the semi-elliptic DOS shifted by -sigma h, closed crosswise
    w = OB.matsubara(beta, n_iw)
    gs = []
    for sigma in (1, -1):
        z = 1j * w + sigma * h
        sq = np.sqrt(z * z - 4.0 * t * t)
        g = (z - sq) / (2.0 * t * t)
        g = np.where(g.imag > 0, (z + sq) / (2.0 * t * t), g)
        gs.append(g)
    return 1.0 / (1j * w - t * t * gs[1]), 1.0 / (1j * w - t * t * gs[0])


def test_af_cycle_u0_semicircle_is_fixed_point(ctx):
    import paper_0801_1222_amd as P
    beta, t = 10.0, 1.0
    b = P.bethe_semicircle_bath(beta, t, 4000)
    out = P.dmft_solve_af(ctx, 0.0, beta, t, [0.5, 0.4, 0.25], 1, 2, b, b, n_chains=2, warmup=1,
                          sweeps=2)
    assert np.abs(out["baths"][0] - b).max() < 1e-10 and np.abs(out["baths"][1] - b).max() < 1e-10
    assert np.abs(out["history"][:, 4]).max() < 1e-12


def test_af_cycle_matches_oracle(ctx):
    import paper_0801_1222_amd as P
    beta, U, t, seed = 4.0, 4.0, 1.0, 7
    dtaus = [0.5, 0.4, 0.25]
    bu, bd = _staggered_baths(beta, t, 0.3, 2000)
    out = P.dmft_solve_af(ctx, U, beta, t, dtaus, seed, 2, bu, bd, n_fine=81, n_chains=3, warmup=5,
                          sweeps=40, mode="rank1")
    ref = OM.dmft_loop_af((bu, bd), U, beta, t, dtaus, seed, 2, n_chains=3, warmup=5, sweeps=40,
                          n_fine=81)
    assert np.abs(out["g"] - ref["g"]).max() < 1e-9
    assert np.abs(out["g_err"] - ref["g_err"]).max() < 1e-9
    assert np.abs(out["baths"][0] - ref["baths"][0]).max() < 1e-9
    assert np.abs(out["baths"][1] - ref["baths"][1]).max() < 1e-9
    assert np.abs(out["history"] - ref["history"]).max() < 1e-9
    # the staggered start is a moment already (its sign is the start's choice)
    assert abs(out["history"][0][4]) > 0.05


def test_neel_order_grows_and_keeps_its_symmetry(ctx):
    import paper_0801_1222_amd as P
    beta, U, t = 20.0, 3.0, 1.0
    dtaus = [beta / L for L in (40, 50, 60, 80)]
    bu, bd = _staggered_baths(beta, t, 0.1, 4096)
    out = P.dmft_solve_af(ctx, U, beta, t, dtaus, 3, 16, bu, bd, n_fine=101, n_chains=64,
                          warmup=50, sweeps=400, mode="delayed", delay_k=16)
    h = out["history"]
    print("moment per iteration", " ".join("%.3f" % m for m in h[:, 4]), flush=True)
    print("D per iteration", " ".join("%.4f" % d for d in h[:, 2]), flush=True)
    m = np.abs(h[:, 4])
    assert m[0] < 0.3 and m[-1] > 0.5 and m[-1] > 2 * m[0]
    assert abs(m[-1] - m[-2]) < 0.05
    g, e = out["g"], out["g_err"]
    # Neel state at half filling: G_dn(tau) = G_up(beta - tau)
    s = np.hypot(e[0][::-1], e[1])
    assert np.all(np.abs(g[1] - g[0][::-1]) < 5 * s + 2e-3)
    assert np.abs(out["baths"][0].real + out["baths"][1].real).max() < 0.05 * np.abs(out["baths"][0]).max()
