// Host numerics shared by the C-ABI entry points (no device code).
#pragma once
#include <vector>

namespace hfqmc {
namespace host {

constexpr double kSigmaFloor = 1e-14;

double matsubara(double beta, int n);
void semicircle(double beta, double t, int n_iw, double* out);
void atomic_seed(double beta, double t, double U, int n_iw, double* out);
void iw_to_tau(const double* f_iw, int n_iw, double m3, double beta, const double* tau, int n_tau,
               double* out, double m2 = 0.0);
void reference_iw(const double* bath_iw, int n_iw, double U, double beta, double* out);
void reference_tau(const double* bath_iw, int n_iw, double m3, double U, double beta,
                   const double* tau, int n_tau, double* out);
void extrapolate(const double* dtaus, int n_grids, const double* g, const double* e, int n_fine,
                 double* c0, double* err);
int bethe_step(const double* g_fine, int n_fine, const double* bath_prev, int n_iw, double m3,
               double U, double beta, double t, double* bath_new);
// away from half filling
void bethe_lattice(double beta, double t, double mu, int n_iw, double* out);
void reference_iw_n(const double* bath_iw, int n_iw, double U, double beta, double n, double* out);
void reference_tau_n(const double* bath_iw, int n_iw, double m2, double m3, double U, double beta,
                     double n, const double* tau, int n_tau, double* out);
int bethe_step_n(const double* g_fine, int n_fine, const double* bath_prev, int n_iw, double m2,
                 double m3, double U, double beta, double t, double mu, double* bath_new);

class Spline {
 public:
  Spline(const double* x, const double* y, int n);
  double operator()(double xq) const;
  void fourier(double beta, int n_iw, double* out) const;

 private:
  void coeffs(int i, double* p) const;
  std::vector<double> x_, y_, m_;
};

}  // namespace host
}  // namespace hfqmc
