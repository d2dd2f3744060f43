"""Hirsch-Fye QMC impurity solver at fixed dtau (oracle side).

TEST INFRASTRUCTURE ONLY: nothing in the product path imports this module.
Plain, slow, FP64 NumPy.  Every function follows the method as the paper
states it (Introduction: Trotter slices of uniform width dtau, a binary
Hubbard-Stratonovich field sampled by Monte Carlo) with the standard
Hirsch-Fye formulas the paper relies on but does not print:

  * Trotter grid            tau_l = l dtau, l = 0..L-1, L = beta / dtau
  * HS coupling             cosh(lambda) = exp(dtau U / 2)
  * potential               V_sigma(l) = lambda sigma s_l,  s_l = +-1
  * bath matrix G0          G0[i, j] = G(tau_{i-j}) for i >= j, -G(tau_{i-j+L}) for i < j
  * Dyson from G0           [1 + (1 - G0)(e^V - 1)] G_sigma = G0
  * flip s_l -> -s_l        gamma_sigma = e^{-2 lambda sigma s_l} - 1
                            R_sigma = 1 + gamma_sigma (1 - G_sigma[l, l]),  R = R_up R_dn
  * rank-1 Dyson update     G <- G + (G[:, l] - e_l) (gamma / R_sigma) G[l, :]
  * measurement             G(tau_k) from translation and spin averaging, D = <n_up n_dn>

Where the paper leaves a point open (matrix sign convention, HS form, sweep
order, acceptance rule, recompute trigger, estimator) the reading taken is the
one stated in the docstring of the function concerned.
"""
import numpy as np

from . import philox


# ---------------------------------------------------------------- set-up ----

def hs_lambda(U, dtau):
    """Hubbard-Stratonovich coupling: cosh(lambda) = exp(dtau U / 2)."""
    return float(np.arccosh(np.exp(0.5 * dtau * U)))


def flip_gammas(lam):
    """(gamma_plus, gamma_minus) = (e^{2 lambda} - 1, e^{-2 lambda} - 1).

    A flip of s_l changes V_sigma(l) by -2 lambda sigma s_l, so spin up uses
    gamma_minus when s_l = +1 and gamma_plus when s_l = -1; spin down the other.
    """
    return float(np.expm1(2.0 * lam)), float(np.expm1(-2.0 * lam))


def g0_matrix(g_tau):
    """Antiperiodic L x L bath matrix from G(tau_k), k = 0..L-1 (G(0) = G(0+))."""
    g_tau = np.asarray(g_tau, dtype=np.float64)
    L = g_tau.shape[0]
    i = np.arange(L)[:, None]
    j = np.arange(L)[None, :]
    d = i - j
    return np.where(d >= 0, g_tau[np.mod(d, L)], -g_tau[np.mod(d, L)])


def potential_factors(s, lam, sigma):
    """e^{V_sigma(l)} - 1 for all slices, V_sigma(l) = lambda sigma s_l."""
    return np.expm1(lam * sigma * np.asarray(s, dtype=np.float64))


def dyson_matrix(G0, s, lam, sigma):
    """M_sigma = 1 + (1 - G0) diag(e^{V_sigma} - 1)."""
    L = G0.shape[0]
    eye = np.eye(L)
    return eye + (eye - G0) * potential_factors(s, lam, sigma)[None, :]


def spin_baths(g_tau):
    """(G0_up(tau_k), G0_dn(tau_k)): a pair as given, or one bath for both spins."""
    if isinstance(g_tau, (tuple, list)) and len(g_tau) == 2 and np.ndim(g_tau[0]) == 1:
        up = np.asarray(g_tau[0], dtype=np.float64)
        dn = np.asarray(g_tau[1], dtype=np.float64)
        if up.shape != dn.shape:
            raise ValueError("spin baths of different lengths")
        return up, dn
    g = np.asarray(g_tau, dtype=np.float64)
    return g, g


def green_from_field(G0, s, lam):
    """Exact G_up, G_dn for field s: solve M_sigma G_sigma = G0_sigma (LU, partial
    pivoting).  G0 is one bath matrix for both spins or a pair (up, down)."""
    G0u, G0d = G0 if isinstance(G0, tuple) else (G0, G0)
    Gu = np.linalg.solve(dyson_matrix(G0u, s, lam, +1), G0u)
    Gd = np.linalg.solve(dyson_matrix(G0d, s, lam, -1), G0d)
    return Gu, Gd


# ---------------------------------------------------------- the update ----

def flip_ratio(Gu_ll, Gd_ll, s_l, gp, gm):
    """Determinant ratio of a proposed flip of s_l, both spins and the product."""
    g_up = gm if s_l > 0 else gp
    g_dn = gp if s_l > 0 else gm
    r_up = 1.0 + g_up * (1.0 - Gu_ll)
    r_dn = 1.0 + g_dn * (1.0 - Gd_ll)
    return g_up, g_dn, r_up, r_dn, r_up * r_dn


def rank1_update(G, l, coef):
    """In place: G <- G + (G[:, l] - e_l) (coef G[l, :]),  coef = gamma / R_sigma."""
    x = G[:, l].copy()
    x[l] -= 1.0
    y = coef * G[l, :]
    G += np.outer(x, y)


# ----------------------------------------------------------- measuring ----

def measure(Gu, Gd):
    """Estimators for one field configuration.

    G(tau_k) = 1/(2L) sum_sigma sum_l sgn G_sigma[(l+k) mod L, l], sgn = -1 when
    l + k wraps past L (antiperiodicity), k = 0..L-1; G(beta-) = 1 - G(0+).
    D = (1/L) sum_l (1 - Gu[l, l]) (1 - Gd[l, l])  (spins decouple at fixed s).
    Returns (g [L+1], D).
    """
    L = Gu.shape[0]
    out = np.empty(L + 1)
    l = np.arange(L)
    for k in range(L):
        r = l + k
        sgn = np.where(r < L, 1.0, -1.0)
        rr = np.mod(r, L)
        out[k] = (np.sum(sgn * Gu[rr, l]) + np.sum(sgn * Gd[rr, l])) / (2.0 * L)
    out[L] = 1.0 - out[0]
    D = float(np.mean((1.0 - np.diag(Gu)) * (1.0 - np.diag(Gd))))
    return out, D


def measure_spins(Gu, Gd):
    """Spin-resolved estimator: G_sigma(tau_k) = 1/L sum_l sgn G_sigma[(l+k) mod L, l],
    G_sigma(beta-) = 1 - G_sigma(0+) = n_sigma.  Returns [2, L+1] (up, down); their
    mean is the estimator of ``measure``."""
    L = Gu.shape[0]
    out = np.empty((2, L + 1))
    l = np.arange(L)
    for k in range(L):
        r = l + k
        sgn = np.where(r < L, 1.0, -1.0)
        rr = np.mod(r, L)
        out[0, k] = np.sum(sgn * Gu[rr, l]) / L
        out[1, k] = np.sum(sgn * Gd[rr, l]) / L
    out[:, L] = 1.0 - out[:, 0]
    return out


# -------------------------------------------------------------- chains ----

def run_chain(g_tau, U, beta, seed, chain=0, grid_id=0, warmup=0, sweeps=1,
              n_rec=100, n_bins=1, replay=None, delay_k=0, flush_fp32=False,
              keep_trace=False, heat_bath=False):
    """One Markov chain of fixed-dtau HF-QMC.

    Sweep order l = 0..L-1; Metropolis acceptance u < R (or, with
    ``heat_bath``, u < R / (1 + R): both satisfy detailed balance for weights
    proportional to det M_up det M_dn) with u from stream 0 of the Philox
    layout; R <= 0 or NaN counts as a reject and is tallied.
    Every ``n_rec`` accepted flips (counted across warm-up) G is recomputed
    from the field and the largest elementwise change is kept as the drift.
    Measurements are taken after every sweep >= warmup.

    ``replay``: optional set of (sweep, l) pairs; when given, a proposal is
    accepted iff it is in the set (its ratio still sets the update).
    ``delay_k`` > 0: delayed updates G_cur = G + A B^T with up to k pending
    vectors, flushed when k are pending, before a recompute and at sweep end;
    ``flush_fp32`` performs that flush as float32 A B^T with float32
    accumulation added to the float64 G (mixed-precision emulation).

    ``g_tau``: one bath for both spins, or a pair (up, down) of spin-dependent
    baths (a magnetic field, magnetic phases); ``bins_gs`` holds the
    spin-resolved sums of ``measure_spins`` either way.

    Returns a dict with the accumulated estimators and bookkeeping.
    """
    g_up, g_dn = spin_baths(g_tau)
    L = g_up.shape[0]
    dtau = beta / L
    lam = hs_lambda(U, dtau)
    gp, gm = flip_gammas(lam)
    G0 = (g0_matrix(g_up), g0_matrix(g_dn))
    s = philox.initial_field(seed, chain, grid_id, L).astype(np.int64)
    Gu, Gd = green_from_field(G0, s, lam)

    bins_g = np.zeros((n_bins, L + 1))
    bins_gs = np.zeros((n_bins, 2, L + 1))
    bins_d = np.zeros(n_bins)
    bins_n = np.zeros(n_bins, dtype=np.int64)
    flips = []
    n_prop = n_acc = n_bad = n_recs = 0
    acc_since = 0
    max_drift = 0.0
    trace = []

    k = int(delay_k)
    if k > 0:
        Au = np.zeros((L, k)); Bu = np.zeros((L, k))
        Ad = np.zeros((L, k)); Bd = np.zeros((L, k))
    m = 0

    def flush():
        nonlocal m
        if k > 0 and m > 0:
            for G, A, B in ((Gu, Au, Bu), (Gd, Ad, Bd)):
                if flush_fp32:
                    prod = np.matmul(A[:, :m].astype(np.float32), B[:, :m].T.astype(np.float32))
                    G += prod.astype(np.float64)
                else:
                    G += A[:, :m] @ B[:, :m].T
            m = 0

    def recompute():
        nonlocal Gu, Gd, max_drift, n_recs
        nu, nd = green_from_field(G0, s, lam)
        drift = max(np.max(np.abs(nu - Gu)), np.max(np.abs(nd - Gd)))
        max_drift = max(max_drift, float(drift))
        Gu[...] = nu
        Gd[...] = nd
        n_recs += 1

    total = warmup + sweeps
    for sw in range(total):
        u = philox.sweep_uniforms(seed, chain, grid_id, sw, L)
        for l in range(L):
            n_prop += 1
            if k > 0 and m > 0:
                gu_ll = Gu[l, l] + Au[l, :m] @ Bu[l, :m]
                gd_ll = Gd[l, l] + Ad[l, :m] @ Bd[l, :m]
            else:
                gu_ll = Gu[l, l]
                gd_ll = Gd[l, l]
            g_up, g_dn, r_up, r_dn, R = flip_ratio(gu_ll, gd_ll, s[l], gp, gm)
            bad = not (R > 0.0)
            if bad:
                n_bad += 1
            if replay is not None:
                accept = (sw, l) in replay
            else:
                accept = (not bad) and (u[l] < (R / (1.0 + R) if heat_bath else R))
            if not accept:
                continue
            n_acc += 1
            flips.append((sw, l))
            if k > 0:
                for G, A, B, g, r in ((Gu, Au, Bu, g_up, r_up), (Gd, Ad, Bd, g_dn, r_dn)):
                    x = G[:, l] + A[:, :m] @ B[l, :m]
                    x[l] -= 1.0
                    y = (g / r) * (G[l, :] + B[:, :m] @ A[l, :m])
                    A[:, m] = x
                    B[:, m] = y
                m += 1
                if m == k:
                    flush()
            else:
                rank1_update(Gu, l, g_up / r_up)
                rank1_update(Gd, l, g_dn / r_dn)
            s[l] = -s[l]
            acc_since += 1
            if acc_since == n_rec:
                flush()
                recompute()
                acc_since = 0
        flush()
        if sw >= warmup:
            g, D = measure(Gu, Gd)
            meas = sw - warmup
            b = (meas * n_bins) // sweeps
            bins_g[b] += g
            bins_gs[b] += measure_spins(Gu, Gd)
            bins_d[b] += D
            bins_n[b] += 1
            if keep_trace:
                trace.append((g, D))
    return dict(L=L, lam=lam, bins_g=bins_g, bins_gs=bins_gs, bins_d=bins_d, bins_n=bins_n,
                flips=flips, n_proposed=n_prop, n_accepted=n_acc, n_bad=n_bad,
                n_recomputes=n_recs, max_drift=max_drift, field=s.copy(),
                Gu=Gu, Gd=Gd, trace=trace)


def reduce_chains(results):
    """Mean and standard error over all (chain, bin) sample means.

    Each chain contributes its bin means (one bin per chain unless a single
    chain is binned); the estimate is their average and the error is their
    sample standard deviation over sqrt(number of samples).
    """
    g_samples = []
    d_samples = []
    for r in results:
        for b in range(r["bins_n"].shape[0]):
            n = r["bins_n"][b]
            if n > 0:
                g_samples.append(r["bins_g"][b] / n)
                d_samples.append(r["bins_d"][b] / n)
    g_samples = np.array(g_samples)
    d_samples = np.array(d_samples)
    ns = g_samples.shape[0]
    g = g_samples.mean(axis=0)
    D = d_samples.mean()
    if ns > 1:
        g_err = g_samples.std(axis=0, ddof=1) / np.sqrt(ns)
        d_err = d_samples.std(ddof=1) / np.sqrt(ns)
    else:
        g_err = np.zeros_like(g)
        d_err = 0.0
    return g, g_err, float(D), float(d_err)


def reduce_chains_spin(results):
    """``reduce_chains`` for the spin-resolved estimator: (G_sigma [2, L+1], its
    error, D, D error) over all (chain, bin) sample means."""
    g_samples, d_samples = [], []
    for r in results:
        for b in range(r["bins_n"].shape[0]):
            n = r["bins_n"][b]
            if n > 0:
                g_samples.append(r["bins_gs"][b] / n)
                d_samples.append(r["bins_d"][b] / n)
    g_samples = np.array(g_samples)
    d_samples = np.array(d_samples)
    ns = g_samples.shape[0]
    g = g_samples.mean(axis=0)
    if ns > 1:
        g_err = g_samples.std(axis=0, ddof=1) / np.sqrt(ns)
        d_err = float(d_samples.std(ddof=1) / np.sqrt(ns))
    else:
        g_err = np.zeros_like(g)
        d_err = 0.0
    return g, g_err, float(d_samples.mean()), d_err


def _chain_job(job):
    """run_chain(*args, **kw) for a (args, kw) pair (a picklable job for process pools)."""
    args, kw = job
    return run_chain(*args, **kw)


def solve(g_tau, U, beta, seed, n_chains=1, warmup=0, sweeps=1, n_rec=100,
          n_bins=None, grid_id=0, mapper=None, **kw):
    """Fixed-dtau solve: n_chains independent chains (chain c uses seed + c).

    ``mapper``: optional map-like callable (e.g. a process pool's ``map``) that
    runs the independent chains; the results are the same as with ``map``.
    """
    if n_bins is None:
        n_bins = 20 if n_chains == 1 else 1
    jobs = [((g_tau, U, beta, seed), dict(chain=c, grid_id=grid_id, warmup=warmup,
                                          sweeps=sweeps, n_rec=n_rec, n_bins=n_bins, **kw))
            for c in range(n_chains)]
    res = list((mapper or map)(_chain_job, jobs))
    g, g_err, D, d_err = reduce_chains(res)
    return dict(g=g, g_err=g_err, D=D, D_err=d_err, chains=res)


# --------------------------------------------------------- brute force ----

def brute_force(g_tau, U, beta, batch=4096, spins=False):
    """Exact fixed-dtau expectation by enumerating all 2^L fields.

    Weight w(s) = det M_up(s) det M_dn(s) (the HS weight up to an s-independent
    factor); returns (G(tau_k) [L+1], D, min weight / max weight), with
    ``spins`` the spin-resolved G_sigma(tau_k) [2, L+1] in place of G.  g_tau:
    one bath or a pair (up, down) as in ``run_chain``.
    """
    g_up, g_dn = spin_baths(g_tau)
    L = g_up.shape[0]
    lam = hs_lambda(U, beta / L)
    G0s = (g0_matrix(g_up), g0_matrix(g_dn))
    eye = np.eye(L)
    n_conf = 1 << L
    logw_all = []
    g_all = []
    d_all = []
    for start in range(0, n_conf, batch):
        idx = np.arange(start, min(start + batch, n_conf))
        bits = (idx[:, None] >> np.arange(L)[None, :]) & 1
        s = np.where(bits == 1, 1.0, -1.0)
        sign_tot = np.ones(idx.shape[0])
        logw = np.zeros(idx.shape[0])
        Gs = []
        for sigma, G0 in ((+1, G0s[0]), (-1, G0s[1])):
            f = np.expm1(lam * sigma * s)
            M = eye[None] + (eye - G0)[None] * f[:, None, :]
            sg, ld = np.linalg.slogdet(M)
            sign_tot *= sg
            logw += ld
            Gs.append(np.linalg.solve(M, np.broadcast_to(G0, M.shape)))
        if np.any(sign_tot <= 0):
            raise ValueError("non-positive HS weight")
        logw_all.append(logw)
        # the estimator of ``measure`` evaluated for the whole batch at once
        l = np.arange(L)
        gb = np.empty((idx.shape[0], 2, L + 1))
        for k in range(L):
            r = l + k
            sgn = np.where(r < L, 1.0, -1.0)
            rr = np.mod(r, L)
            gb[:, 0, k] = (Gs[0][:, rr, l] * sgn).sum(axis=1) / L
            gb[:, 1, k] = (Gs[1][:, rr, l] * sgn).sum(axis=1) / L
        gb[:, :, L] = 1.0 - gb[:, :, 0]
        du = np.diagonal(Gs[0], axis1=1, axis2=2)
        dd = np.diagonal(Gs[1], axis1=1, axis2=2)
        g_all.append(gb)
        d_all.append(np.mean((1.0 - du) * (1.0 - dd), axis=1))
    logw = np.concatenate(logw_all)
    w = np.exp(logw - logw.max())
    g_all = np.concatenate(g_all)
    d_all = np.concatenate(d_all)
    Z = w.sum()
    gs = np.tensordot(w, g_all, axes=(0, 0)) / Z
    return (gs if spins else gs.mean(axis=0)), float((w * d_all).sum() / Z), float(w.min())


# ---------------------------------------------------------- closed forms ----

def atomic_limit_g(U, beta, tau):
    """Half-filled Hubbard atom: G(tau) = cosh((beta/2 - tau) U/2) / (2 cosh(beta U / 4))."""
    tau = np.asarray(tau, dtype=np.float64)
    return np.cosh((0.5 * beta - tau) * 0.5 * U) / (2.0 * np.cosh(0.25 * beta * U))


def atomic_limit_d(U, beta):
    """Half-filled Hubbard atom: D = 1 / (2 (1 + e^{beta U / 2}))."""
    return 1.0 / (2.0 * (1.0 + np.exp(0.5 * beta * U)))


# ------------------------------------------ an atomic level at any filling ----
# The bath of an isolated level eps0 (chemical potential -eps0) and the exact
# Green function and double occupancy of the Hubbard atom built on it.  The
# interaction is the decoupled U (n_up n_dn - (n_up + n_dn)/2); the four states
# have energies 0, E1 = eps0 - U/2 (twice), E2 = 2 eps0.  HF-QMC is
# Trotter-exact here for every L (everything is diagonal in the occupations).

def atomic_level_bath(eps0, beta, tau):
    """G0(tau) = e^{-eps0 tau} / (1 + e^{-beta eps0}), 0 <= tau < beta (positive convention)."""
    tau = np.asarray(tau, dtype=np.float64)
    return np.exp(-eps0 * tau) / (1.0 + np.exp(-beta * eps0))


def atomic_level_g(eps0, U, beta, tau):
    """G(tau) = [e^{-tau E1} + e^{-beta E1} e^{-tau (E2 - E1)}] / Z, Z = 1 + 2 e^{-beta E1} + e^{-beta E2}."""
    tau = np.asarray(tau, dtype=np.float64)
    e1, e2 = eps0 - 0.5 * U, 2.0 * eps0
    z = 1.0 + 2.0 * np.exp(-beta * e1) + np.exp(-beta * e2)
    return (np.exp(-tau * e1) + np.exp(-beta * e1) * np.exp(-tau * (e2 - e1))) / z


def atomic_level_d(eps0, U, beta):
    """D = e^{-beta E2} / Z."""
    e1, e2 = eps0 - 0.5 * U, 2.0 * eps0
    z = 1.0 + 2.0 * np.exp(-beta * e1) + np.exp(-beta * e2)
    return np.exp(-beta * e2) / z


# ------------------------------------------- the atom in a magnetic field ----
# Spin-dependent levels eps_up, eps_dn (a Zeeman splitting): the four states
# have energies 0, E_up = eps_up - U/2, E_dn = eps_dn - U/2, E2 = eps_up + eps_dn;
# again Trotter-exact for every L.

def atomic_field_g(eps_up, eps_dn, U, beta, tau):
    """(G_up(tau), G_dn(tau)): G_sigma = [e^{-tau E_sigma} + e^{-beta E_-sigma}
    e^{-tau (E2 - E_-sigma)}] / Z, Z = 1 + e^{-beta E_up} + e^{-beta E_dn} + e^{-beta E2}."""
    tau = np.asarray(tau, dtype=np.float64)
    eu, ed, e2 = eps_up - 0.5 * U, eps_dn - 0.5 * U, eps_up + eps_dn
    z = 1.0 + np.exp(-beta * eu) + np.exp(-beta * ed) + np.exp(-beta * e2)
    gu = (np.exp(-tau * eu) + np.exp(-beta * ed) * np.exp(-tau * (e2 - ed))) / z
    gd = (np.exp(-tau * ed) + np.exp(-beta * eu) * np.exp(-tau * (e2 - eu))) / z
    return gu, gd


def atomic_field_d(eps_up, eps_dn, U, beta):
    """D = e^{-beta E2} / Z."""
    eu, ed, e2 = eps_up - 0.5 * U, eps_dn - 0.5 * U, eps_up + eps_dn
    z = 1.0 + np.exp(-beta * eu) + np.exp(-beta * ed) + np.exp(-beta * e2)
    return np.exp(-beta * e2) / z
