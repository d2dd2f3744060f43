"""Multigrid step and Bethe-lattice DMFT step (oracle side).

TEST INFRASTRUCTURE ONLY: nothing in the product path imports this module.

The multigrid HF-QMC method (section "Multigrid HF-QMC method", Fig. 1(c))
solves the impurity problem at a fixed bath for several dtau_i, then
  (i)  interpolates each discrete estimate G_dtau_i(tau_k) onto a common fine
       tau grid with the help of a reference model, and
  (ii) performs, on that grid, a least-squares fit that is quadratic in
       dtau^2 and keeps its dtau -> 0 value.
The paper delegates the details of (i) to other work; the readings taken here:
  * reference model  G_ref(i w) = 1 / (1/Bath(i w) - U^2 / (4 i w)), the
    half-filled atomic self-energy on top of the bath.  It has the exact
    1/(i w)^3 moment (m3 + U^2/4) and reproduces U = 0 and the atomic limit;
  * interpolation    natural cubic spline of G_i - G_ref through all L_i + 1
    points tau_k = k beta / L_i (tau_L = beta-), plus G_ref on the fine grid;
    errors are interpolated linearly;
  * extrapolation    weighted least squares G_i = c0 + c1 x_i + c2 x_i^2,
    x_i = dtau_i^2, weights 1/sigma_i^2 (sigma floored at SIGMA_FLOOR); the
    result is c0 with error sqrt([(X^T W X)^{-1}]_00).
The DMFT closure for the Bethe lattice with hopping t (semi-elliptic DOS,
W = 4t) is Bath_new(i w) = 1/(i w - t^2 G(i w)), with G(i w) obtained as
G_ref(i w) plus the exact Fourier integral of the cubic spline of G - G_ref.
"""
import numpy as np
from scipy.interpolate import CubicSpline

from . import bath as B
from . import hfqmc as H

SIGMA_FLOOR = 1e-14


def reference_iw(bath_iw, U, beta):
    """Reference model on the Matsubara axis."""
    w = B.matsubara(beta, bath_iw.shape[0])
    return 1.0 / (1.0 / bath_iw - U * U / (4.0 * 1j * w))


def reference_tau(bath_iw, m3, U, beta, tau):
    """Reference model at imaginary times (tail moment m3 + U^2/4)."""
    return B.iw_to_tau(reference_iw(bath_iw, U, beta), m3 + 0.25 * U * U, beta, tau)


def grid_lengths(beta, dtaus):
    """Trotter numbers L_i = round(beta / dtau_i); the exact dtau_i = beta / L_i is used."""
    Ls = [int(round(beta / d)) for d in dtaus]
    return Ls, [beta / L for L in Ls]


def fine_grid(beta, n_fine):
    """Common fine grid tau_j = j beta / (n_fine - 1), endpoints included (tau = beta-)."""
    return np.arange(n_fine) * (beta / (n_fine - 1))


def interpolate_grid(g_grid, err_grid, beta, gref_grid, gref_fine, tau_fine):
    """Step (i): spline G_i - G_ref over tau_k = k beta / L, add G_ref back."""
    L = g_grid.shape[0] - 1
    tau_k = np.arange(L + 1) * (beta / L)
    cs = CubicSpline(tau_k, g_grid - gref_grid, bc_type="natural")
    g_f = gref_fine + cs(tau_fine)
    e_f = np.interp(tau_fine, tau_k, err_grid)
    return g_f, e_f


def extrapolate(dtaus, g_interp, e_interp):
    """Step (ii): per fine point, weighted quadratic-in-dtau^2 least squares.

    g_interp, e_interp: [n_grids, n_fine].  Returns (c0 [n_fine], err [n_fine]).
    """
    x = np.asarray(dtaus, dtype=np.float64) ** 2
    X = np.stack([np.ones_like(x), x, x * x], axis=1)
    n_fine = g_interp.shape[1]
    c0 = np.empty(n_fine)
    err = np.empty(n_fine)
    for j in range(n_fine):
        sig = np.maximum(e_interp[:, j], SIGMA_FLOOR)
        w = 1.0 / sig ** 2
        A = X.T @ (w[:, None] * X)
        b = X.T @ (w * g_interp[:, j])
        cov = np.linalg.inv(A)
        coef = cov @ b
        c0[j] = coef[0]
        err[j] = np.sqrt(max(cov[0, 0], 0.0))
    return c0, err


def multigrid_solve(bath_iw, m3, U, beta, dtaus, seed, n_chains, warmup, sweeps,
                    n_rec=100, n_fine=200, mapper=None):
    """Oracle multigrid solve: one fixed-dtau solve per grid (grid_id = i), then (i), (ii).

    ``mapper``: optional map-like callable running each grid's independent chains
    (see ``hfqmc.solve``); it does not change the result."""
    Ls, dts = grid_lengths(beta, dtaus)
    tau_f = fine_grid(beta, n_fine)
    gref_f = reference_tau(bath_iw, m3, U, beta, tau_f)
    gi, ei, per = [], [], []
    for i, L in enumerate(Ls):
        g_tau = B.bath_to_tau(bath_iw, m3, beta, L)
        r = H.solve(g_tau, U, beta, seed, n_chains=n_chains, warmup=warmup,
                    sweeps=sweeps, n_rec=n_rec, grid_id=i, mapper=mapper)
        tau_k = np.arange(L + 1) * (beta / L)
        gref_k = reference_tau(bath_iw, m3, U, beta, tau_k)
        g_f, e_f = interpolate_grid(r["g"], r["g_err"], beta, gref_k, gref_f, tau_f)
        gi.append(g_f)
        ei.append(e_f)
        per.append(r)
    c0, err = extrapolate(dts, np.array(gi), np.array(ei))
    # the double occupancy D(dtau^2) of each grid (the quantity of Figs. 3 and 4),
    # extrapolated by the same weighted quadratic fit
    d_g = np.array([[r["D"]] for r in per])
    d_e = np.array([[r["D_err"]] for r in per])
    d0, d0e = extrapolate(dts, d_g, d_e)
    return dict(g=c0, g_err=err, tau=tau_f, grids=per, g_interp=np.array(gi),
                e_interp=np.array(ei), Ls=Ls, dtaus=dts, D=float(d0[0]), D_err=float(d0e[0]))


def multigrid_solve_spin(baths, m3, U, beta, dtaus, seed, n_chains, warmup, sweeps,
                         n_rec=100, n_fine=200):
    """Multigrid solve with spin-dependent baths (up, down): one spin-resolved
    fixed-dtau solve per grid, then steps (i) and (ii) for each spin with that
    spin's reference model.  g: [2, n_fine] (up, down); g_interp: [n_grids, 2, n_fine]."""
    Ls, dts = grid_lengths(beta, dtaus)
    tau_f = fine_grid(beta, n_fine)
    n_bins = 20 if n_chains == 1 else 1
    gref_f = [reference_tau(b, m3, U, beta, tau_f) for b in baths]
    gi, ei, d_g, d_e = [], [], [], []
    for i, L in enumerate(Ls):
        g_taus = tuple(B.bath_to_tau(b, m3, beta, L) for b in baths)
        res = [H.run_chain(g_taus, U, beta, seed, chain=c, grid_id=i, warmup=warmup,
                           sweeps=sweeps, n_rec=n_rec, n_bins=n_bins) for c in range(n_chains)]
        gs, gs_err, D, D_err = H.reduce_chains_spin(res)
        tau_k = np.arange(L + 1) * (beta / L)
        gf, ef = [], []
        for sp in (0, 1):
            gref_k = reference_tau(baths[sp], m3, U, beta, tau_k)
            a, e = interpolate_grid(gs[sp], gs_err[sp], beta, gref_k, gref_f[sp], tau_f)
            gf.append(a)
            ef.append(e)
        gi.append(gf)
        ei.append(ef)
        d_g.append([D])
        d_e.append([D_err])
    gi = np.array(gi)
    ei = np.array(ei)
    g = np.empty((2, n_fine))
    g_err = np.empty((2, n_fine))
    for sp in (0, 1):
        g[sp], g_err[sp] = extrapolate(dts, gi[:, sp], ei[:, sp])
    d0, d0e = extrapolate(dts, np.array(d_g), np.array(d_e))
    return dict(g=g, g_err=g_err, tau=tau_f, g_interp=gi, e_interp=ei, Ls=Ls, dtaus=dts,
                D=float(d0[0]), D_err=float(d0e[0]))


# ------------------------------------------------ away from half filling ----
# The method applies at any filling (closing remarks); the readings taken:
#   * the bath's tail 1/(i w) + m2/(i w)^2 + m3/(i w)^3 (bath.iw_to_tau);
#   * reference model at density n per spin: G_ref = 1/(1/Bath - Sigma_ref) with
#     the first two high-frequency terms of the self-energy of the interaction
#     U (n_up n_dn - (n_up + n_dn)/2), Sigma_ref(i w) = U (n - 1/2) + U^2 n (1 - n)/(i w)
#     (n = 1/2: the half-filled reference above); G_ref's tail moments follow
#     from the bath's;
#   * n of the interpolation: the estimate G(beta-) of the finest grid; n of the
#     closure's transform: the extrapolated G(beta-);
#   * Bethe closure at chemical potential mu (from half filling):
#     Bath = 1/(i w + mu - t^2 G), tail moments m2 = -mu, m3 = mu^2 + t^2.

def reference_iw_n(bath_iw, U, beta, n):
    """Reference model at density n per spin on the Matsubara axis."""
    iw = 1j * B.matsubara(beta, bath_iw.shape[0])
    return 1.0 / (1.0 / bath_iw - U * (n - 0.5) - U * U * n * (1.0 - n) / iw)


def reference_moments(m2, m3, U, n):
    """(M2, M3) of G_ref = 1/(1/Bath - s0 - s1/(i w)), Bath ~ 1/(i w) + m2/(i w)^2 + m3/(i w)^3:
    1/Bath = i w - m2 + (m2^2 - m3)/(i w) + ..., so M2 = m2 + s0 and
    M3 = M2^2 - (m2^2 - m3 - s1), with s0 = U (n - 1/2), s1 = U^2 n (1 - n)."""
    s0 = U * (n - 0.5)
    s1 = U * U * n * (1.0 - n)
    M2 = m2 + s0
    return M2, M2 * M2 - (m2 * m2 - m3 - s1)


def reference_tau_n(bath_iw, m2, m3, U, beta, tau, n):
    """Reference model at density n at imaginary times."""
    M2, M3 = reference_moments(m2, m3, U, n)
    return B.iw_to_tau(reference_iw_n(bath_iw, U, beta, n), M3, beta, tau, m2=M2)


def multigrid_solve_n(bath_iw, m2, m3, U, beta, dtaus, seed, n_chains, warmup, sweeps,
                      n_rec=100, n_fine=200, mapper=None):
    """Multigrid solve at any filling: one fixed-dtau solve per grid (grid_id = i, the bath
    with its 1/(i w)^2 moment m2), then steps (i) and (ii) with the reference model at
    the finest grid's density n = G(beta-)."""
    Ls, dts = grid_lengths(beta, dtaus)
    tau_f = fine_grid(beta, n_fine)
    per = []
    for i, L in enumerate(Ls):
        g_tau = B.bath_to_tau(bath_iw, m3, beta, L, m2=m2)
        per.append(H.solve(g_tau, U, beta, seed, n_chains=n_chains, warmup=warmup,
                           sweeps=sweeps, n_rec=n_rec, grid_id=i, mapper=mapper))
    n_ref = float(per[int(np.argmax(Ls))]["g"][-1])
    gref_f = reference_tau_n(bath_iw, m2, m3, U, beta, tau_f, n_ref)
    gi, ei = [], []
    for L, r in zip(Ls, per):
        tau_k = np.arange(L + 1) * (beta / L)
        gref_k = reference_tau_n(bath_iw, m2, m3, U, beta, tau_k, n_ref)
        g_f, e_f = interpolate_grid(r["g"], r["g_err"], beta, gref_k, gref_f, tau_f)
        gi.append(g_f)
        ei.append(e_f)
    c0, err = extrapolate(dts, np.array(gi), np.array(ei))
    d0, d0e = extrapolate(dts, np.array([[r["D"]] for r in per]),
                          np.array([[r["D_err"]] for r in per]))
    return dict(g=c0, g_err=err, tau=tau_f, grids=per, g_interp=np.array(gi),
                e_interp=np.array(ei), Ls=Ls, dtaus=dts, D=float(d0[0]), D_err=float(d0e[0]),
                n_ref=n_ref)


def dmft_bethe_step_n(g_fine, tau_fine, bath_iw, m2, m3, U, beta, t, mu):
    """Closure at chemical potential mu: G(i w) = G_ref(i w) - FT[spline(G - G_ref)] with the
    reference at the density n = G(beta-) of g_fine, then 1/(i w + mu - t^2 G(i w))."""
    n = float(g_fine[-1])
    gref_f = reference_tau_n(bath_iw, m2, m3, U, beta, tau_fine, n)
    delta = spline_fourier(tau_fine, np.asarray(g_fine) - gref_f, beta, bath_iw.shape[0])
    g_iw = reference_iw_n(bath_iw, U, beta, n) - delta
    return B.bethe_step_iw(g_iw, beta, t, mu=mu)


def dmft_loop_mu(bath_iw, U, mu, beta, t, dtaus, seed, n_iter, n_chains, warmup, sweeps,
                 n_rec=100, n_fine=200, mixing=0.0):
    """The DMFT cycle of Fig. 1(c) at chemical potential mu on the Bethe lattice: the
    bath keeps the tail moments m2 = -mu, m3 = mu^2 + t^2.  history[it] = (max |g -
    g_prev|, max g_err, D, D_err, n), n = G(beta-) extrapolated."""
    m2, m3 = -mu, mu * mu + t * t
    bath = np.asarray(bath_iw, dtype=np.complex128).copy()
    tau_f = fine_grid(beta, n_fine)
    prev = reference_tau_n(bath, m2, m3, 0.0, beta, tau_f, 0.5)   # U = 0: the bath itself
    hist = []
    r = None
    for it in range(n_iter):
        r = multigrid_solve_n(bath, m2, m3, U, beta, dtaus, seed + (it << 32), n_chains, warmup,
                              sweeps, n_rec=n_rec, n_fine=n_fine)
        hist.append((float(np.abs(r["g"] - prev).max()), float(r["g_err"].max()), r["D"],
                     r["D_err"], float(r["g"][-1])))
        prev = r["g"]
        new = dmft_bethe_step_n(r["g"], tau_f, bath, m2, m3, U, beta, t, mu)
        bath = mixing * bath + (1.0 - mixing) * new
    return dict(bath=bath, g=r["g"], g_err=r["g_err"], tau=tau_f, history=np.array(hist))


def spline_fourier(tau, values, beta, n_iw):
    """Exact int_0^beta e^{i w_n tau} S(tau) d tau for the natural cubic spline S.

    On each interval the integral of e^{i w tau} p(tau) for a cubic p is
    [e^{i w tau} sum_{m=0}^{3} (-1)^m p^{(m)}(tau) / (i w)^{m+1}] between its ends.
    """
    cs = CubicSpline(tau, values, bc_type="natural")
    c = cs.c  # c[m, i]: coefficient of (tau - tau_i)^(3-m)
    h = np.diff(tau)
    a3, a2, a1, a0 = c[0], c[1], c[2], c[3]
    # derivatives at the left ends
    dl = [a0, a1, 2 * a2, 6 * a3]
    # derivatives at the right ends
    dr = [a0 + a1 * h + a2 * h ** 2 + a3 * h ** 3,
          a1 + 2 * a2 * h + 3 * a3 * h ** 2,
          2 * a2 + 6 * a3 * h,
          6 * a3]
    w = B.matsubara(beta, n_iw)
    iw = 1j * w
    out = np.zeros(n_iw, dtype=np.complex128)
    for m in range(4):
        coef = (-1.0) ** m / iw ** (m + 1)
        right = np.exp(1j * np.outer(w, tau[1:])) @ dr[m]
        left = np.exp(1j * np.outer(w, tau[:-1])) @ dl[m]
        out += coef * (right - left)
    return out


def g_tau_to_iw(g_fine, tau_fine, bath_iw, m3, U, beta):
    """G(i w) = G_ref(i w) - FT[spline(G - G_ref)] (positive tau convention)."""
    gref_f = reference_tau(bath_iw, m3, U, beta, tau_fine)
    delta = spline_fourier(tau_fine, np.asarray(g_fine) - gref_f, beta, bath_iw.shape[0])
    return reference_iw(bath_iw, U, beta) - delta


def dmft_bethe_step(g_fine, tau_fine, bath_iw, m3, U, beta, t):
    """One Bethe-lattice self-consistency step: the new bath on the same frequencies."""
    g_iw = g_tau_to_iw(g_fine, tau_fine, bath_iw, m3, U, beta)
    return B.bethe_step_iw(g_iw, beta, t)


def dmft_loop(bath_iw, U, beta, t, dtaus, seed, n_iter, n_chains, warmup, sweeps, n_rec=100,
              n_fine=200, mixing=0.0, ph=False):
    """The DMFT cycle of Fig. 1(c) on the Bethe lattice, n_iter times: a multigrid
    impurity solve at the current bath (fresh random streams per iteration: the
    seed moves by 2^32), then the closure Bath_new = 1/(i w - t^2 G(i w)), mixed
    as mixing * old + (1 - mixing) * new.  The bath's 1/(i w)^3 moment stays t^2.
    history[it] = (max |g - g_prev|, max g_err, D, D_err), g_prev of the first
    iteration being the starting bath's own G0(tau_j), D the extrapolated double
    occupancy.  With ph (a particle-hole symmetric cycle) the new bath keeps
    only its imaginary part: the transform of a symmetric G(tau) has none, and
    the rounding left there is magnified by an insulating bath's pole near
    zero frequency."""
    m3 = t * t
    bath = np.asarray(bath_iw, dtype=np.complex128).copy()
    tau_f = fine_grid(beta, n_fine)
    prev = reference_tau(bath, m3, 0.0, beta, tau_f)
    hist = []
    r = None
    for it in range(n_iter):
        r = multigrid_solve(bath, m3, U, beta, dtaus, seed + (it << 32), n_chains, warmup, sweeps,
                            n_rec=n_rec, n_fine=n_fine)
        hist.append((float(np.abs(r["g"] - prev).max()), float(r["g_err"].max()), r["D"],
                     r["D_err"]))
        prev = r["g"]
        new = dmft_bethe_step(r["g"], r["tau"], bath, m3, U, beta, t)
        if ph:
            new = 1j * new.imag
        bath = mixing * bath + (1.0 - mixing) * new
    return dict(bath=bath, g=r["g"], g_err=r["g_err"], tau=tau_f, history=np.array(hist))


def dmft_loop_af(baths, U, beta, t, dtaus, seed, n_iter, n_chains, warmup, sweeps, n_rec=100,
                 n_fine=200, mixing=0.0):
    """The DMFT cycle for Neel order on the bipartite Bethe lattice: sublattice B
    is sublattice A with the spins exchanged, so spin sigma's new bath closes
    over the other spin's Green function, Bath_sigma = 1/(i w - t^2 G_-sigma(i w))
    (the paper's closing remarks on magnetic phases; Fig. 1(c) otherwise).
    history[it] = (max |g - g_prev| over both spins, max g_err, D, D_err,
    m = n_up - n_dn), n_sigma = G_sigma(beta-) extrapolated."""
    m3 = t * t
    bu = np.asarray(baths[0], dtype=np.complex128).copy()
    bd = np.asarray(baths[1], dtype=np.complex128).copy()
    tau_f = fine_grid(beta, n_fine)
    prev = np.array([reference_tau(bu, m3, 0.0, beta, tau_f), reference_tau(bd, m3, 0.0, beta, tau_f)])
    hist = []
    r = None
    for it in range(n_iter):
        r = multigrid_solve_spin((bu, bd), m3, U, beta, dtaus, seed + (it << 32), n_chains, warmup,
                                 sweeps, n_rec=n_rec, n_fine=n_fine)
        g = r["g"]
        hist.append((float(np.abs(g - prev).max()), float(r["g_err"].max()), r["D"], r["D_err"],
                     float(g[0, -1] - g[1, -1])))
        prev = g
        new_dn = dmft_bethe_step(g[0], tau_f, bu, m3, U, beta, t)
        new_up = dmft_bethe_step(g[1], tau_f, bd, m3, U, beta, t)
        bu = mixing * bu + (1.0 - mixing) * new_up
        bd = mixing * bd + (1.0 - mixing) * new_dn
    return dict(baths=(bu, bd), g=r["g"], g_err=r["g_err"], tau=tau_f, history=np.array(hist))
