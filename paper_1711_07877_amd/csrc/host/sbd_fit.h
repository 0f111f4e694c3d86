// Off-line SBD fit on the host in FP64 (Sections 2-5 of the paper).
#pragma once
#include <complex>
#include <cstdint>
#include <string>
#include <vector>

namespace sbd {

struct FitResult {
  int kind = 0;            // 0 Laplace, 1 Helmholtz, 2 general
  double a = 0;            // annulus inner radius of the fitted shape (Helmholtz: lambda * a)
  int P = 0;
  double lam = 1.0;        // J0 argument dilation (Helmholtz lambda = kappa / kappa')
  double kappa = 0, kappa_p = 0;
  double robin_H = 0;      // > 0: Dini basis of the Robin condition u' + H u = 0 (no rescaling)
  double err = 0;          // max error on the check grid
  std::vector<double> rho, C, alpha;
  std::vector<double> coef;    // alpha_p C_p: coefficient of J0(rho_p lam s)
  std::vector<double> radii;   // rho_p lam (unit-scaled circle radii)
  std::vector<int64_t> M;      // nodes per circle
  // Helmholtz: the J0(kappa s) part as one exact circle.
  double extra_radius = 0;
  int64_t extra_M = 0;
  // General kernel: P counts the fitted circles and then the n enforced ones
  // (radii omega_t, coef mu_t); rho, C, alpha hold the fitted P - n only.
  int n_enforced = 0;
  double constant = 0;         // G_SBD = constant + sum_p coef_p J0(radii_p s)
};

// General radial kernel G(r) = c_log log r + sum_j r^m_j (a_j sin(w_j r) + b_j cos(w_j r)).
struct TrigTerm {
  int m;
  double w, a, b;
};
struct GeneralKernel {
  double c_log = 0;
  std::vector<TrigTerm> terms;
  int enforce = 0;             // multi-Dirichlet order n
};
double general_eval(const GeneralKernel& g, double r);

// Fit of the unit-scaled shape g(s) = G(delta_max s) on [a, 1] with the
// multi-Dirichlet condition enforced to order g.enforce (Section 4.3).
int sbd_fit_general(const GeneralKernel& g, double delta_max, double a, double eps, int nthreads,
                    FitResult& out, std::string& msg);

// Status codes follow sbd_status (0 ok, -4 floor, -1 invalid).
int sbd_fit(int kind, double a, double eps, double kappa, int force_P, int nthreads,
            FitResult& out, std::string& msg);

// Circle size rule: smallest even M > x with 2 (|J_M(x)| + |J_2M(x)|) <= eta.
int64_t circle_size(double x, double eta);

// Chebyshev tables for the close-correction values on u = r^2 in [0, U]:
//   D(u) = A(u) log(u) + B(u)   (u > 0),  D(0) = self (diagonal, complex).
struct NearTables {
  int deg = 0;
  double U = 0;
  std::vector<double> A, B;    // Chebyshev coefficients on t = 2u/U - 1
  std::complex<double> self;
};
// For the general kernel (kind 2) B is a Chebyshev series in r = sqrt(u) on [0, sqrt(U)]
// (its odd powers of r are not smooth in u), A is the constant c_log / 2.
NearTables near_tables(const FitResult& fit, int kind, double delta_max, double U, double wavenumber,
                       int deg, const GeneralKernel* gk = nullptr);

// G_SBD(r) of the plan (radial series, un-scaled), complex for Helmholtz.
std::complex<double> g_sbd(const FitResult& fit, int kind, double delta_max, double wavenumber, double r);

// Chebyshev coefficients (degree deg) of the 1-D Fourier transform of the
// exponential-of-semicircle kernel phi(x) = exp(beta (sqrt(1 - (x/alpha)^2) - 1)),
// phi_hat(t) = int phi(x) cos(t x) dx, on t in [0, tmax] (mapped to [-1, 1]).
std::vector<double> es_hat_cheb(double beta, double alpha, double tmax, int deg);
double es_hat(double beta, double alpha, double t);

}  // namespace sbd
