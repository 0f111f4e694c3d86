#include "bessel.h"

#include <cmath>
#include <limits>

namespace sbd {
namespace bessel {

namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr double kEulerGamma = 0.57721566490153286061;

// Backward recurrence: fills J_0..J_nmax(x) (x > 0, x <= ~60).
void miller(double x, int nmax, std::vector<double>& out) {
  int start = nmax + 20 + static_cast<int>(x + 12.0 * std::cbrt(x + 1.0));
  if (start % 2) ++start;
  out.assign(nmax + 1, 0.0);
  double jp1 = 0.0, jcur = 1e-300, norm = 0.0;
  for (int k = start; k > 0; --k) {
    double jm1 = (2.0 * k / x) * jcur - jp1;   // J_{k-1}
    jp1 = jcur;
    jcur = jm1;
    // now jcur = J_{k-1}
    int n = k - 1;
    if (n <= nmax) out[n] = jcur;
    if (n > 0 && (n % 2 == 0)) norm += 2.0 * jcur;
    if (std::fabs(jcur) > 1e250) {  // rescale to avoid overflow
      jp1 *= 1e-250; jcur *= 1e-250; norm *= 1e-250;
      for (double& v : out) v *= 1e-250;
    }
  }
  norm += jcur;  // J_0
  for (double& v : out) v /= norm;
}

// Hankel asymptotic sums P_nu, Q_nu for large x (DLMF 10.17.3): returns P, Q with
// J_nu = sqrt(2/(pi x)) (P cos w - Q sin w), Y_nu = sqrt(2/(pi x)) (P sin w + Q cos w).
void hankel_pq(int nu, double x, double* P, double* Q) {
  double mu = 4.0 * nu * nu;
  double ak = 1.0;  // a_0
  double p = 1.0, q = 0.0, xp = 1.0;
  double prev = 1e300;
  for (int k = 1; k < 60; ++k) {
    ak *= (mu - (2.0 * k - 1) * (2.0 * k - 1)) / (8.0 * k);
    xp *= x;
    double term = ak / xp;
    if (std::fabs(term) > prev) break;  // asymptotic series: stop at smallest term
    prev = std::fabs(term);
    // k odd -> Q gets (-1)^((k-1)/2) term; k even -> P gets (-1)^(k/2) term
    if (k % 2 == 1) q += ((k / 2) % 2 ? -term : term);
    else p += ((k / 2) % 2 ? -term : term);
    if (prev < 1e-18) break;
  }
  *P = p;
  *Q = q;
}

}  // namespace

void j0j1(double x, double* J0, double* J1) {
  x = std::fabs(x);
  if (x == 0.0) { *J0 = 1.0; *J1 = 0.0; return; }
  if (x <= kSmallArg) {
    std::vector<double> v;
    miller(x, 1, v);
    *J0 = v[0];
    *J1 = v[1];
    return;
  }
  double s = std::sin(x), c = std::cos(x);
  double amp = std::sqrt(2.0 / (kPi * x));
  double P, Q;
  hankel_pq(0, x, &P, &Q);
  // w = x - pi/4: cos w = (c + s)/sqrt2, sin w = (s - c)/sqrt2
  const double r2 = 0.70710678118654752440;
  double cw = (c + s) * r2, sw = (s - c) * r2;
  *J0 = amp * (P * cw - Q * sw);
  hankel_pq(1, x, &P, &Q);
  // w = x - 3pi/4: cos w = (s - c)/sqrt2, sin w = (s + c)/sqrt2... sin(x-3pi/4) = -(s + c)/sqrt2? check:
  // cos(x - 3pi/4) = cos x cos 3pi/4 + sin x sin 3pi/4 = (-c + s)/sqrt2
  // sin(x - 3pi/4) = sin x cos 3pi/4 - cos x sin 3pi/4 = (-s - c)/sqrt2
  cw = (s - c) * r2;
  sw = -(s + c) * r2;
  *J1 = amp * (P * cw - Q * sw);
}

double j0(double x) { double a, b; j0j1(x, &a, &b); return a; }
double j1(double x) {
  double a, b;
  j0j1(x, &a, &b);
  return x < 0 ? -b : b;
}

static void y0y1(double x, double* Y0, double* Y1) {
  if (x <= kSmallArg) {
    int nmax = static_cast<int>(x) + 60;
    std::vector<double> J;
    miller(x, nmax, J);
    double L = std::log(0.5 * x) + kEulerGamma;
    double s0 = 0.0, s1 = 0.0;
    for (int k = 1; 2 * k + 1 <= nmax; ++k) {
      double sg = (k % 2) ? -1.0 : 1.0;
      s0 += sg * J[2 * k] / k;
      s1 += sg * (J[2 * k - 1] - J[2 * k + 1]) / k;
    }
    *Y0 = (2.0 / kPi) * L * J[0] - (4.0 / kPi) * s0;
    *Y1 = -(2.0 / kPi) * J[0] / x + (2.0 / kPi) * L * J[1] + (2.0 / kPi) * s1;
    return;
  }
  double s = std::sin(x), c = std::cos(x);
  double amp = std::sqrt(2.0 / (kPi * x));
  const double r2 = 0.70710678118654752440;
  double P, Q;
  hankel_pq(0, x, &P, &Q);
  double cw = (c + s) * r2, sw = (s - c) * r2;
  *Y0 = amp * (P * sw + Q * cw);
  hankel_pq(1, x, &P, &Q);
  cw = (s - c) * r2;
  sw = -(s + c) * r2;
  *Y1 = amp * (P * sw + Q * cw);
}

double y0(double x) { double a, b; y0y1(x, &a, &b); return a; }
double y1(double x) { double a, b; y0y1(x, &a, &b); return b; }

double jn_small(int n, double x) {
  if (x == 0.0) return n == 0 ? 1.0 : 0.0;
  std::vector<double> v;
  miller(x, n, v);
  return v[n];
}

double log_abs_jn_tail(double nu, double x) {
  if (x <= 0.0) return -std::numeric_limits<double>::infinity();
  if (x <= 50.0 && nu <= 400.0) {
    double v = std::fabs(jn_small(static_cast<int>(nu), x));
    return v > 0 ? std::log(v) : -745.0;
  }
  if (nu - x < 2.0 * std::cbrt(nu)) return std::numeric_limits<double>::infinity();
  // x = nu sech(a); Debye: J_nu ~ e^{nu (tanh a - a)} / sqrt(2 pi nu tanh a) (1 + u1/nu + u2/nu^2)
  double sech = x / nu;
  double a = std::acosh(1.0 / sech);
  double th = std::tanh(a);
  double p = 1.0 / th;
  double u1 = (3.0 * p - 5.0 * p * p * p) / 24.0;
  double p2 = p * p;
  double u2 = (81.0 * p2 - 462.0 * p2 * p2 + 385.0 * p2 * p2 * p2) / 1152.0;
  double corr = 1.0 + std::fabs(u1) / nu + std::fabs(u2) / (nu * nu);
  return nu * (th - a) - 0.5 * std::log(2.0 * kPi * nu * th) + std::log(corr);
}

static double mcmahon(double beta) {
  double b = 8.0 * beta;
  double b2 = b * b;
  // nu = 0 (mu = 0): beta + 1/(8 beta) - 4*31/(3 (8beta)^3) + 32*3779/(15 (8beta)^5) ...
  return beta + 1.0 / b - 124.0 / (3.0 * b * b2) + 120928.0 / (15.0 * b * b2 * b2);
}

std::vector<double> j0_zeros(int n) {
  std::vector<double> z(n);
  for (int m = 1; m <= n; ++m) {
    double x = mcmahon((m - 0.25) * kPi);
    for (int it = 0; it < 8; ++it) {
      double a, b;
      j0j1(x, &a, &b);
      double dx = a / b;  // x_new = x - J0/J0' = x + J0/J1
      x += dx;
      if (std::fabs(dx) < 1e-15 * x) break;
    }
    z[m - 1] = x;
  }
  return z;
}

std::vector<double> y0_zeros(int n) {
  std::vector<double> z(n);
  for (int m = 1; m <= n; ++m) {
    double x = mcmahon((m - 0.75) * kPi);
    for (int it = 0; it < 12; ++it) {
      double a, b;
      y0y1(x, &a, &b);
      double dx = a / b;
      x += dx;
      if (std::fabs(dx) < 1e-15 * x) break;
    }
    z[m - 1] = x;
  }
  return z;
}

double y0_zero_at_least(double x) {
  int m = static_cast<int>(std::floor(x / kPi + 0.75)) - 1;
  if (m < 1) m = 1;
  auto z = y0_zeros(m + 3);
  for (double v : z)
    if (v >= x) return v;
  return z.back();
}

}  // namespace bessel
}  // namespace sbd
