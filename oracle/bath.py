"""Bath Green functions for the Bethe lattice (oracle side).

TEST INFRASTRUCTURE ONLY: nothing in the product path imports this module.

The paper's benchmark model is the one-band Hubbard model with a semi-elliptic
density of states of bandwidth W = 4 (Benchmark results section), i.e. hopping
t = 1 on the Bethe lattice.  The impurity bath enters Hirsch-Fye QMC only
through its imaginary-time values on the Trotter grid tau_k = k * dtau.

Conventions (the paper is silent on them; the readings are listed in the design notes):
  * Matsubara functions use the standard sign, F(i w_n) ~ 1/(i w_n), with
    w_n = (2n+1) pi / beta, n >= 0 stored, F(-i w) = conj F(i w).
  * Imaginary-time functions use the "positive" convention
    G(tau) = <T c(tau) c^dag(0)>, 0 < tau < beta, so G(0+) = 1 - n = 1/2 at
    half filling and G(beta-) = n.
"""
import numpy as np


def matsubara(beta, n_iw):
    """Fermionic Matsubara frequencies w_n = (2n+1) pi / beta, n = 0..n_iw-1."""
    return (2.0 * np.arange(n_iw) + 1.0) * np.pi / beta


def semicircle_iw(beta, t, n_iw):
    """Local Green function of the Bethe lattice with half-bandwidth 2t at i w_n.

    G(z) = (z - sqrt(z^2 - 4 t^2)) / (2 t^2), branch with G ~ 1/z; at z = i w
    this is i (w - sgn(w) sqrt(w^2 + 4 t^2)) / (2 t^2).  This is the U = 0 bath
    and the starting point of the self-consistency cycle (Fig. 1).
    """
    w = matsubara(beta, n_iw)
    return 1j * (w - np.sqrt(w * w + 4.0 * t * t)) / (2.0 * t * t)


def iw_to_tau(f_iw, m3, beta, tau, m2=0.0):
    """Positive-convention G(tau) at 0 <= tau < beta (tau = 0 means 0+).

    Fourier sum over the stored frequencies with the known high-frequency tail
    1/(i w) + m2/(i w)^2 + m3/(i w)^3 subtracted and added back in closed form
    ((1/beta) sum over all n of e^{-i w_n tau} / (i w_n)^p is -1/2, (2 tau -
    beta)/4 and tau (beta - tau)/4 for p = 1, 2, 3):
      G_std(tau) = -1/2 + m2 (2 tau - beta)/4 + m3 tau (beta - tau)/4
                   + (2/beta) sum_n Re[e^{-i w_n tau} (F - 1/(i w) - m2/(i w)^2 - m3/(i w)^3)]
      G_pos(tau) = -G_std(tau).
    m2 = 0 for a particle-hole symmetric function (half filling).
    """
    f_iw = np.asarray(f_iw, dtype=np.complex128)
    tau = np.atleast_1d(np.asarray(tau, dtype=np.float64))
    w = matsubara(beta, f_iw.shape[0])
    iw = 1j * w
    rem = f_iw - 1.0 / iw - m2 / iw ** 2 - m3 / iw ** 3
    out = np.empty(tau.shape[0])
    for a in range(tau.shape[0]):
        s = np.sum((np.exp(-1j * w * tau[a]) * rem).real)
        g_std = (-0.5 + m2 * (2.0 * tau[a] - beta) / 4.0 + m3 * tau[a] * (beta - tau[a]) / 4.0
                 + 2.0 / beta * s)
        out[a] = -g_std
    return out


def bath_to_tau(bath_iw, m3, beta, L, m2=0.0):
    """Bath on a Trotter grid: G(tau_k), tau_k = k beta / L, k = 0..L-1."""
    tau = np.arange(L) * (beta / L)
    return iw_to_tau(bath_iw, m3, beta, tau, m2=m2)


def semicircle_tau_dos(beta, t, tau, n_nodes=20000, mu=0.0):
    """Independent route: G(tau) = int rho(e) e^{-tau (e - mu)} / (1 + e^{-beta (e - mu)}) de.

    rho(e) = sqrt(4t^2 - e^2) / (2 pi t^2); with e = 2 t x this is
    (2/pi) int_{-1}^{1} sqrt(1 - x^2) f(2 t x) dx, evaluated by Gauss-Chebyshev
    quadrature of the second kind.  Used only to pin ``iw_to_tau``.
    """
    i = np.arange(1, n_nodes + 1)
    th = i * np.pi / (n_nodes + 1)
    x = np.cos(th)
    wts = np.pi / (n_nodes + 1) * np.sin(th) ** 2
    e = 2.0 * t * x - mu
    tau = np.atleast_1d(np.asarray(tau, dtype=np.float64))
    out = np.empty(tau.shape[0])
    for a in range(tau.shape[0]):
        ta = tau[a]
        pos = e >= 0
        f = np.empty_like(e)
        f[pos] = np.exp(-ta * e[pos]) / (1.0 + np.exp(-beta * e[pos]))
        f[~pos] = np.exp((beta - ta) * e[~pos]) / (1.0 + np.exp(beta * e[~pos]))
        out[a] = 2.0 / np.pi * np.sum(wts * f)
    return out


def bethe_step_iw(g_iw, beta, t, mu=0.0):
    """Bethe-lattice closure of the DMFT cycle: new bath 1/(i w + mu - t^2 G(i w)).

    mu is the chemical potential measured from half filling (the interaction
    U (n_up n_dn - (n_up + n_dn)/2) of the symmetric decoupling carries the
    Hartree shift of the half-filled case).  The new bath's tail is
    1/(i w) - mu/(i w)^2 + (mu^2 + t^2)/(i w)^3 whatever G is."""
    w = matsubara(beta, g_iw.shape[0])
    return 1.0 / (1j * w + mu - t * t * np.asarray(g_iw))


def bethe_lattice_iw(beta, t, mu, n_iw):
    """Noninteracting local Green function of the Bethe lattice at chemical
    potential mu: G(z) = (z - sqrt(z - 2t) sqrt(z + 2t)) / (2 t^2), z = i w + mu
    (principal square roots: the branch with G ~ 1/z and Im G < 0), evaluated
    as 2 / (z + sqrt(z - 2t) sqrt(z + 2t)), the same number without the
    cancellation at large |z|.  At U = 0 it solves the closure G = 1/(z - t^2 G):
    the fixed point of the cycle."""
    z = 1j * matsubara(beta, n_iw) + mu
    return 2.0 / (z + np.sqrt(z - 2.0 * t) * np.sqrt(z + 2.0 * t))


def bethe_lattice_iw_dos(beta, t, mu, n_iw, n_nodes=20000):
    """Independent route: G(i w) = int rho(e) / (i w + mu - e) de with the
    semi-elliptic rho(e) = sqrt(4t^2 - e^2)/(2 pi t^2), by the Gauss-Chebyshev
    quadrature of semicircle_tau_dos.  Used only to pin ``bethe_lattice_iw``."""
    i = np.arange(1, n_nodes + 1)
    th = i * np.pi / (n_nodes + 1)
    x = np.cos(th)
    wts = np.pi / (n_nodes + 1) * np.sin(th) ** 2
    e = 2.0 * t * x
    z = 1j * matsubara(beta, n_iw) + mu
    return 2.0 / np.pi * (wts[None, :] / (z[:, None] - e[None, :])).sum(axis=1)


def atomic_seed_iw(beta, t, U, n_iw):
    """Insulating starting bath: the Bethe closure applied to the half-filled
    Hubbard atom, 1/(i w - t^2 G_at(i w)) with
    G_at(i w) = (1/(i w - U/2) + 1/(i w + U/2)) / 2.

    The atomic Green function has a Mott gap of width U; seeding the DMFT
    cycle with it leads to the insulating solution where metal and insulator
    coexist (Benchmark results section, Fig. 3).  Its 1/(i w)^3 moment is t^2,
    like that of the semicircle.  At U = 0 it is the bath of a bare level.
    """
    iw = 1j * matsubara(beta, n_iw)
    g_at = 0.5 * (1.0 / (iw - 0.5 * U) + 1.0 / (iw + 0.5 * U))
    return bethe_step_iw(g_at, beta, t)
