// Host-side numerics around the device hot path: bath transforms, the two
// multigrid steps and the Bethe-lattice closure of the DMFT cycle.
//
// Section "Multigrid HF-QMC method" of the paper: each discrete HF-QMC
// estimate G_dtau_i is (i) interpolated onto a common fine tau grid with the
// help of a reference model and (ii) extrapolated to dtau -> 0 by a
// least-squares fit quadratic in dtau^2.  Readings taken where the paper
// defers to other work: reference model 1/(1/bath - U^2/(4 i w)); natural
// cubic spline of G - G_ref through all L+1 grid points (tau_L = beta-);
// errors interpolated linearly; weights 1/sigma^2 with sigma floored at 1e-14;
// Bethe closure bath_new = 1/(i w - t^2 G(i w)) (Fig. 1, W = 4t).
#include "hfqmc_host.h"

#include <cmath>
#include <complex>
#include <vector>

namespace hfqmc {
namespace host {

using cd = std::complex<double>;

double matsubara(double beta, int n) { return (2.0 * n + 1.0) * M_PI / beta; }

void semicircle(double beta, double t, int n_iw, double* out) {
  for (int n = 0; n < n_iw; ++n) {
    const double w = matsubara(beta, n);
    // G(i w) = i (w - sqrt(w^2 + 4 t^2)) / (2 t^2)
    out[2 * n] = 0.0;
    out[2 * n + 1] = (w - std::sqrt(w * w + 4.0 * t * t)) / (2.0 * t * t);
  }
}

// Bethe closure of the half-filled Hubbard atom, 1/(i w - t^2 G_at(i w)):
// G_at(i w) = i w / ((i w)^2 - U^2/4) = -i w / (w^2 + U^2/4), so the bath is
// -i / (w (1 + t^2 / (w^2 + U^2/4))), purely imaginary like the semicircle.
void atomic_seed(double beta, double t, double U, int n_iw, double* out) {
  const double a = 0.25 * U * U;
  for (int n = 0; n < n_iw; ++n) {
    const double w = matsubara(beta, n);
    out[2 * n] = 0.0;
    out[2 * n + 1] = -1.0 / (w * (1.0 + t * t / (w * w + a)));
  }
}

// Positive-convention G(tau) from Matsubara data with the tail
// 1/(i w) + m2/(i w)^2 + m3/(i w)^3 summed in closed form:
//   G_std(tau) = -1/2 + m2 (2 tau - beta)/4 + m3 tau (beta - tau)/4
//                + (2/beta) sum_n Re[e^{-i w tau} rem_n]
// (m2 = 0 at half filling).
void iw_to_tau(const double* f_iw, int n_iw, double m3, double beta, const double* tau, int n_tau,
               double* out, double m2) {
  std::vector<double> rr(n_iw), ri(n_iw), w(n_iw);
  for (int n = 0; n < n_iw; ++n) {
    w[n] = matsubara(beta, n);
    const cd iw(0.0, w[n]);
    const cd f(f_iw[2 * n], f_iw[2 * n + 1]);
    const cd rem = f - 1.0 / iw - m2 / (iw * iw) - m3 / (iw * iw * iw);
    rr[n] = rem.real();
    ri[n] = rem.imag();
  }
  for (int a = 0; a < n_tau; ++a) {
    const double ta = tau[a];
    double s = 0.0;
    for (int n = 0; n < n_iw; ++n) {
      // Re[(cos - i sin)(rr + i ri)] = cos rr + sin ri
      const double ph = w[n] * ta;
      s += std::cos(ph) * rr[n] + std::sin(ph) * ri[n];
    }
    const double g_std =
        -0.5 + m2 * (2.0 * ta - beta) / 4.0 + m3 * ta * (beta - ta) / 4.0 + 2.0 / beta * s;
    out[a] = -g_std;
  }
}

void reference_iw(const double* bath_iw, int n_iw, double U, double beta, double* out) {
  for (int n = 0; n < n_iw; ++n) {
    const cd iw(0.0, matsubara(beta, n));
    const cd b(bath_iw[2 * n], bath_iw[2 * n + 1]);
    const cd r = 1.0 / (1.0 / b - U * U / (4.0 * iw));
    out[2 * n] = r.real();
    out[2 * n + 1] = r.imag();
  }
}

void reference_tau(const double* bath_iw, int n_iw, double m3, double U, double beta,
                   const double* tau, int n_tau, double* out) {
  std::vector<double> r(2 * (size_t)n_iw);
  reference_iw(bath_iw, n_iw, U, beta, r.data());
  iw_to_tau(r.data(), n_iw, m3 + 0.25 * U * U, beta, tau, n_tau, out);
}

// Natural cubic spline through (x_i, y_i): second derivatives from the
// standard tridiagonal system with M_0 = M_{n-1} = 0.
Spline::Spline(const double* x, const double* y, int n) : x_(x, x + n), y_(y, y + n), m_(n, 0.0) {
  if (n < 3) return;
  std::vector<double> a(n, 0.0), b(n, 1.0), c(n, 0.0), d(n, 0.0);
  for (int i = 1; i < n - 1; ++i) {
    const double h0 = x[i] - x[i - 1], h1 = x[i + 1] - x[i];
    a[i] = h0 / 6.0;
    b[i] = (h0 + h1) / 3.0;
    c[i] = h1 / 6.0;
    d[i] = (y[i + 1] - y[i]) / h1 - (y[i] - y[i - 1]) / h0;
  }
  // Thomas algorithm on rows 1..n-2 (rows 0 and n-1 fix M = 0)
  for (int i = 2; i < n - 1; ++i) {
    const double f = a[i] / b[i - 1];
    b[i] -= f * c[i - 1];
    d[i] -= f * d[i - 1];
  }
  for (int i = n - 2; i >= 1; --i) m_[i] = (d[i] - (i + 1 < n - 1 ? c[i] * m_[i + 1] : 0.0)) / b[i];
}

// Polynomial coefficients of interval i in powers of (x - x_i): p0..p3.
void Spline::coeffs(int i, double* p) const {
  const double h = x_[i + 1] - x_[i];
  p[0] = y_[i];
  p[1] = (y_[i + 1] - y_[i]) / h - h * (2.0 * m_[i] + m_[i + 1]) / 6.0;
  p[2] = m_[i] / 2.0;
  p[3] = (m_[i + 1] - m_[i]) / (6.0 * h);
}

double Spline::operator()(double xq) const {
  const int n = (int)x_.size();
  int lo = 0, hi = n - 1;
  if (xq <= x_[0]) {
    hi = 1;
  } else if (xq >= x_[n - 1]) {
    lo = n - 2;
  } else {
    while (hi - lo > 1) {
      const int mid = (lo + hi) / 2;
      if (x_[mid] <= xq)
        lo = mid;
      else
        hi = mid;
    }
  }
  double p[4];
  coeffs(lo, p);
  const double dx = xq - x_[lo];
  return p[0] + dx * (p[1] + dx * (p[2] + dx * p[3]));
}

// int_0^beta e^{i w tau} S(tau) d tau, exactly, for the spline S: on each
// interval [e^{i w tau} sum_m (-1)^m S^(m)(tau) / (i w)^{m+1}] between its ends.
void Spline::fourier(double beta, int n_iw, double* out) const {
  const int n = (int)x_.size();
  for (int q = 0; q < n_iw; ++q) {
    const double w = matsubara(beta, q);
    const cd iw(0.0, w);
    cd inv[4];
    inv[0] = 1.0 / iw;
    for (int m = 1; m < 4; ++m) inv[m] = inv[m - 1] / iw;
    cd acc(0.0, 0.0);
    for (int i = 0; i + 1 < n; ++i) {
      double p[4];
      coeffs(i, p);
      const double h = x_[i + 1] - x_[i];
      const double dl[4] = {p[0], p[1], 2.0 * p[2], 6.0 * p[3]};
      const double dr[4] = {p[0] + h * (p[1] + h * (p[2] + h * p[3])),
                            p[1] + h * (2.0 * p[2] + 3.0 * h * p[3]), 2.0 * p[2] + 6.0 * h * p[3],
                            6.0 * p[3]};
      const cd el = std::exp(cd(0.0, w * x_[i]));
      const cd er = std::exp(cd(0.0, w * x_[i + 1]));
      for (int m = 0; m < 4; ++m) {
        const double sg = (m & 1) ? -1.0 : 1.0;
        acc += sg * inv[m] * (er * dr[m] - el * dl[m]);
      }
    }
    out[2 * q] = acc.real();
    out[2 * q + 1] = acc.imag();
  }
}

// Step (ii): per point, weighted least squares c0 + c1 x + c2 x^2, x = dtau^2.
void extrapolate(const double* dtaus, int n_grids, const double* g, const double* e, int n_fine,
                 double* c0, double* err) {
  for (int j = 0; j < n_fine; ++j) {
    double A[3][3] = {{0}}, b[3] = {0};
    for (int i = 0; i < n_grids; ++i) {
      const double x = dtaus[i] * dtaus[i];
      const double row[3] = {1.0, x, x * x};
      double sg = e[(size_t)i * n_fine + j];
      if (sg < kSigmaFloor) sg = kSigmaFloor;
      const double w = 1.0 / (sg * sg);
      for (int r = 0; r < 3; ++r) {
        b[r] += row[r] * w * g[(size_t)i * n_fine + j];
        for (int c = 0; c < 3; ++c) A[r][c] += row[r] * w * row[c];
      }
    }
    // inverse of the symmetric 3x3 normal matrix by cofactors
    const double c00 = A[1][1] * A[2][2] - A[1][2] * A[2][1];
    const double c01 = A[0][2] * A[2][1] - A[0][1] * A[2][2];
    const double c02 = A[0][1] * A[1][2] - A[0][2] * A[1][1];
    const double det = A[0][0] * c00 + A[1][0] * c01 + A[2][0] * c02;
    const double inv00 = c00 / det, inv01 = c01 / det, inv02 = c02 / det;
    c0[j] = inv00 * b[0] + inv01 * b[1] + inv02 * b[2];
    err[j] = inv00 > 0.0 ? std::sqrt(inv00) : 0.0;
  }
}

int bethe_step(const double* g_fine, int n_fine, const double* bath_prev, int n_iw, double m3,
               double U, double beta, double t, double* bath_new) {
  std::vector<double> tau(n_fine), gref(n_fine), diff(n_fine);
  for (int j = 0; j < n_fine; ++j) tau[j] = j * (beta / (n_fine - 1));
  reference_tau(bath_prev, n_iw, m3, U, beta, tau.data(), n_fine, gref.data());
  for (int j = 0; j < n_fine; ++j) diff[j] = g_fine[j] - gref[j];
  Spline sp(tau.data(), diff.data(), n_fine);
  std::vector<double> ft(2 * (size_t)n_iw), ref(2 * (size_t)n_iw);
  sp.fourier(beta, n_iw, ft.data());
  reference_iw(bath_prev, n_iw, U, beta, ref.data());
  for (int q = 0; q < n_iw; ++q) {
    const cd iw(0.0, matsubara(beta, q));
    const cd G = cd(ref[2 * q], ref[2 * q + 1]) - cd(ft[2 * q], ft[2 * q + 1]);
    const cd nb = 1.0 / (iw - t * t * G);
    bath_new[2 * q] = nb.real();
    bath_new[2 * q + 1] = nb.imag();
  }
  return 0;
}

// ---------------------------------------------- away from half filling ----
// The closing remarks of the paper state the method's generality; the readings
// for other fillings: the bath's tail carries a 1/(i w)^2 moment m2; the Bethe
// closure has a chemical potential mu measured from half filling,
// bath = 1/(i w + mu - t^2 G) (tail moments -mu, mu^2 + t^2); the reference
// model at density n per spin is 1/(1/bath - s0 - s1/(i w)) with the first two
// high-frequency terms of the self-energy of U (n_up n_dn - (n_up + n_dn)/2),
// s0 = U (n - 1/2) and s1 = U^2 n (1 - n), which at n = 1/2 is the half-filled
// reference above.

// Noninteracting Bethe-lattice G at chemical potential mu, z = i w + mu:
// (z - sqrt(z - 2t) sqrt(z + 2t)) / (2 t^2), principal roots (G ~ 1/z), written
// 2 / (z + sqrt(z - 2t) sqrt(z + 2t)) to avoid the cancellation at large |z|.
void bethe_lattice(double beta, double t, double mu, int n_iw, double* out) {
  for (int n = 0; n < n_iw; ++n) {
    const cd z(mu, matsubara(beta, n));
    const cd g = 2.0 / (z + std::sqrt(z - 2.0 * t) * std::sqrt(z + 2.0 * t));
    out[2 * n] = g.real();
    out[2 * n + 1] = g.imag();
  }
}

void reference_iw_n(const double* bath_iw, int n_iw, double U, double beta, double n, double* out) {
  const double s0 = U * (n - 0.5), s1 = U * U * n * (1.0 - n);
  for (int q = 0; q < n_iw; ++q) {
    const cd iw(0.0, matsubara(beta, q));
    const cd b(bath_iw[2 * q], bath_iw[2 * q + 1]);
    const cd r = 1.0 / (1.0 / b - s0 - s1 / iw);
    out[2 * q] = r.real();
    out[2 * q + 1] = r.imag();
  }
}

// With 1/bath = i w - m2 + (m2^2 - m3)/(i w) + ..., the reference's tail moments
// are M2 = m2 + s0 and M3 = M2^2 - (m2^2 - m3 - s1).
void reference_tau_n(const double* bath_iw, int n_iw, double m2, double m3, double U, double beta,
                     double n, const double* tau, int n_tau, double* out) {
  const double s0 = U * (n - 0.5), s1 = U * U * n * (1.0 - n);
  const double M2 = m2 + s0;
  const double M3 = M2 * M2 - (m2 * m2 - m3 - s1);
  std::vector<double> r(2 * (size_t)n_iw);
  reference_iw_n(bath_iw, n_iw, U, beta, n, r.data());
  iw_to_tau(r.data(), n_iw, M3, beta, tau, n_tau, out, M2);
}

// The closure at mu: G(i w) = G_ref(i w) - FT[spline(G - G_ref)], the reference at
// the density n = G(beta-) of g_fine, then 1/(i w + mu - t^2 G(i w)).
int bethe_step_n(const double* g_fine, int n_fine, const double* bath_prev, int n_iw, double m2,
                 double m3, double U, double beta, double t, double mu, double* bath_new) {
  const double n = g_fine[n_fine - 1];
  std::vector<double> tau(n_fine), gref(n_fine), diff(n_fine);
  for (int j = 0; j < n_fine; ++j) tau[j] = j * (beta / (n_fine - 1));
  reference_tau_n(bath_prev, n_iw, m2, m3, U, beta, n, tau.data(), n_fine, gref.data());
  for (int j = 0; j < n_fine; ++j) diff[j] = g_fine[j] - gref[j];
  Spline sp(tau.data(), diff.data(), n_fine);
  std::vector<double> ft(2 * (size_t)n_iw), ref(2 * (size_t)n_iw);
  sp.fourier(beta, n_iw, ft.data());
  reference_iw_n(bath_prev, n_iw, U, beta, n, ref.data());
  for (int q = 0; q < n_iw; ++q) {
    const cd iw(0.0, matsubara(beta, q));
    const cd G = cd(ref[2 * q], ref[2 * q + 1]) - cd(ft[2 * q], ft[2 * q + 1]);
    const cd nb = 1.0 / (iw + mu - t * t * G);
    bath_new[2 * q] = nb.real();
    bath_new[2 * q + 1] = nb.imag();
  }
  return 0;
}

}  // namespace host
}  // namespace hfqmc
