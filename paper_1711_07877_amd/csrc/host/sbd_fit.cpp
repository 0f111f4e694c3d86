// Off-line SBD fit (host, FP64).
//
//  * Basis (Section 2.1): rho_p zeros of J0, e_p = C_p J0(rho_p r),
//    C_p = 1 / (sqrt(pi) rho_p |J1(rho_p)|).
//  * Fit (Section 3.1/3.2): minimise the H^1 seminorm of the error on the
//    annulus a < r < 1 by A^P alpha = b with the explicit Gram matrix A^P.
//    The off-diagonal bracket follows from Green's formula,
//      int_a^1 r u' v' dr = rho_i rho_j [F_ji - F_ij]_a^1 / (rho_j^2 - rho_i^2),
//    F_ij(r) = rho_i r J0(rho_i r) J0'(rho_j r); the printed formula carries the
//    opposite sign (a misprint; the derivation and quadrature agree here).
//  * Order P: one Cholesky factor of A at an upper order serves every smaller
//    order (leading principal blocks), so the dichotomy of Section 1 costs one
//    factorisation plus O(P^2) per trial; the error is monitored on 4096
//    points clustered near a (where it peaks, Section 4.1 remark).
//  * Circles (Section 5, eq. "temp1"): per-circle budget eps/(2 P |alpha_p C_p|)
//    against the exact aliasing tail 2(|J_M| + |J_2M|) of the M-point rule.
//  * Helmholtz (Section 4.2): Y0(kappa s) through Y0(kappa' t), kappa' the
//    next Y0 zero, fitted on [lambda a, 1]; J0(kappa s) is one exact circle.
//    Below the first zero of Y0 (where lambda would shrink the annulus and
//    lengthen the series) Y0(kappa s) is fitted on [a, 1] in the Dini basis of
//    the Robin condition u' + H u = 0, H = kappa Y1(kappa) / Y0(kappa) > 0
//    (Section 2.3): rho_p the positive roots of H J0(r) - r J1(r), e_p normalised
//    in a_H(u, v) = int_B grad u . grad v + H int_C u v, and the fit minimises
//    a_H of the error on the annulus (Gram and right-hand side gain the boundary
//    terms 2 pi H e_i(1) e_j(1) and 2 pi H G(1) e_j(1)).
#include "sbd_fit.h"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <map>
#include <thread>
#include <tuple>

#include "bessel.h"

namespace sbd {

namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr int kNCheck = 4096;

template <typename F>
void parallel_for(int64_t n, int nthreads, F&& f, int64_t chunk = 1) {
  if (nthreads <= 1 || n <= chunk) {
    for (int64_t i = 0; i < n; ++i) f(i);
    return;
  }
  std::atomic<int64_t> next{0};
  std::vector<std::thread> th;
  for (int t = 0; t < nthreads; ++t)
    th.emplace_back([&] {
      for (;;) {
        int64_t s = next.fetch_add(chunk);
        if (s >= n) break;
        int64_t e = std::min(n, s + chunk);
        for (int64_t i = s; i < e; ++i) f(i);
      }
    });
  for (auto& x : th) x.join();
}

inline double dot(const double* a, const double* b, int n) {
  double s0 = 0, s1 = 0, s2 = 0, s3 = 0;
  int i = 0;
  for (; i + 4 <= n; i += 4) {
    s0 += a[i] * b[i];
    s1 += a[i + 1] * b[i + 1];
    s2 += a[i + 2] * b[i + 2];
    s3 += a[i + 3] * b[i + 3];
  }
  for (; i < n; ++i) s0 += a[i] * b[i];
  return (s0 + s1) + (s2 + s3);
}

// Blocked right-looking Cholesky, row-major, lower triangle.  false if not SPD.
bool cholesky(std::vector<double>& A, int n, int nthreads) {
  const int nb = 96;
  for (int kb = 0; kb < n; kb += nb) {
    int e = std::min(n, kb + nb);
    for (int j = kb; j < e; ++j) {
      double* Aj = &A[(size_t)j * n];
      double d = Aj[j] - dot(Aj + kb, Aj + kb, j - kb);
      if (!(d > 0)) return false;
      Aj[j] = std::sqrt(d);
      for (int i = j + 1; i < e; ++i) {
        double* Ai = &A[(size_t)i * n];
        Ai[j] = (Ai[j] - dot(Ai + kb, Aj + kb, j - kb)) / Aj[j];
      }
    }
    // panel rows below the block
    parallel_for(n - e, nthreads, [&](int64_t ii) {
      int i = e + (int)ii;
      double* Ai = &A[(size_t)i * n];
      for (int j = kb; j < e; ++j) {
        const double* Aj = &A[(size_t)j * n];
        Ai[j] = (Ai[j] - dot(Ai + kb, Aj + kb, j - kb)) / Aj[j];
      }
    }, 32);
    // trailing update of the lower triangle, A22 -= L21 L21^T, as a tiled product: the
    // panel L21 is packed k-major once (LT[k][j - e]), then each task updates the rows of
    // one 64-row block against one 32-column block, a row at a time with 32 running sums
    // over the panel width (contiguous in j, so they vectorise)
    const int w = e - kb;
    const int m = n - e;
    if (m <= 0) continue;
    std::vector<double> LT((size_t)w * m);
    parallel_for(m, nthreads, [&](int64_t jj) {
      const double* Aj = &A[(size_t)(e + jj) * n + kb];
      for (int k = 0; k < w; ++k) LT[(size_t)k * m + jj] = Aj[k];
    }, 256);
    constexpr int MB = 64, NB = 32;
    const int nbi = (m + MB - 1) / MB;
    std::vector<std::pair<int, int>> tiles;
    for (int bi = 0; bi < nbi; ++bi)
      for (int bj = 0; bj * NB < std::min(m, (bi + 1) * MB); ++bj) tiles.emplace_back(bi, bj);
    parallel_for((int64_t)tiles.size(), nthreads, [&](int64_t t) {
      const int i0 = tiles[t].first * MB, j0 = tiles[t].second * NB;
      const int i1 = std::min(m, i0 + MB), j1 = std::min(m, j0 + NB);
      const bool full = j1 - j0 == NB;
      for (int ii = std::max(i0, j0); ii < i1; ++ii) {
        const double* Li = &A[(size_t)(e + ii) * n + kb];
        double acc[NB] = {0};
        if (full) {
          for (int k = 0; k < w; ++k) {
            const double a = Li[k];
            const double* lt = &LT[(size_t)k * m + j0];
#pragma GCC unroll 32
            for (int jj = 0; jj < NB; ++jj) acc[jj] += a * lt[jj];
          }
        } else {
          for (int k = 0; k < w; ++k) {
            const double a = Li[k];
            const double* lt = &LT[(size_t)k * m + j0];
            for (int jj = 0; jj < j1 - j0; ++jj) acc[jj] += a * lt[jj];
          }
        }
        double* Ci = &A[(size_t)(e + ii) * n + e];
        const int jend = std::min(j1, ii + 1);  // lower triangle only
        for (int jj = j0; jj < jend; ++jj) Ci[jj] -= acc[jj - j0];
      }
    }, 1);
  }
  return true;
}

// Radial functions sum c r^m sin(W r) or c r^m cos(W r), keyed (m, W, 1 sin / 0 cos):
// closed under d/dr and 1/r, which is all the iterated Laplacians need.
using TrigKey = std::tuple<int, double, int>;
using TrigMap = std::map<TrigKey, double>;

// d/dr of f + c_log log r
TrigMap trig_d(const TrigMap& f, double c_log) {
  TrigMap out;
  for (const auto& kv : f) {
    const int m = std::get<0>(kv.first);
    const double W = std::get<1>(kv.first);
    const int sn = std::get<2>(kv.first);
    const double c = kv.second;
    if (c == 0.0) continue;
    if (m != 0) out[TrigKey{m - 1, W, sn}] += c * m;
    if (W != 0.0) {
      if (sn) out[TrigKey{m, W, 0}] += c * W;
      else out[TrigKey{m, W, 1}] -= c * W;
    }
  }
  if (c_log != 0.0) out[TrigKey{-1, 0.0, 0}] += c_log;
  return out;
}

// -(f'' + f'/r): minus the radial Laplacian (log r is harmonic away from 0)
TrigMap trig_neg_lap(const TrigMap& f) {
  TrigMap d1 = trig_d(f, 0.0);
  TrigMap out = trig_d(d1, 0.0);
  for (const auto& kv : d1) out[TrigKey{std::get<0>(kv.first) - 1, std::get<1>(kv.first), std::get<2>(kv.first)}] += kv.second;
  for (auto& kv : out) kv.second = -kv.second;
  return out;
}

double trig_eval(const TrigMap& f, double r) {
  double v = 0.0;
  for (const auto& kv : f) {
    const double W = std::get<1>(kv.first);
    const double t = std::get<2>(kv.first) ? std::sin(W * r) : std::cos(W * r);
    v += kv.second * std::pow(r, std::get<0>(kv.first)) * t;
  }
  return v;
}

// H = g - K of the general kernel on the unit-scaled interval: g(s) = G(delta_max s) =
// c log delta_max + c log s + T(s), K(s) = sum_t mu_t J0(omega_t s).
struct GenShape {
  double c = 0;                    // coefficient of log s
  double clogd = 0;                // c log delta_max
  TrigMap T, dT;                   // trigonometric part of g and its derivative
  std::vector<double> om, mu;
  double H1 = 0;                   // (H - c log delta_max) at s = 1
  double wmax = 0;                 // largest frequency of T and K
  double h(double s) const {       // H(s) - c log delta_max
    double v = (c != 0.0 ? c * std::log(s) : 0.0) + trig_eval(T, s);
    for (size_t t = 0; t < om.size(); ++t) v -= mu[t] * bessel::j0(om[t] * s);
    return v;
  }
  double dh_smooth(double s) const {  // H'(s) - c / s
    double v = trig_eval(dT, s);
    for (size_t t = 0; t < om.size(); ++t) v += mu[t] * om[t] * bessel::j1(om[t] * s);
    return v;
  }
};

struct Problem {
  int kind;
  double a;        // fit interval [a, 1]
  double kp;       // Helmholtz kappa' (the Dini fit: kappa itself)
  double H = 0;    // > 0: Dini basis of the Robin condition with this constant
  const GenShape* gen = nullptr;   // kind 2
};

double target(const Problem& pb, double t) {
  if (pb.kind == 2) return pb.gen->h(t) - pb.gen->H1;   // the Dirichlet basis vanishes at 1
  return pb.kind == 0 ? std::log(t) : bessel::y0(pb.kp * t);
}

// 16-point Gauss-Legendre rule on [-1, 1]: Newton's method on P_16 from the
// Chebyshev-like initial guesses, weights 2 / ((1 - x^2) P_16'(x)^2).
void gauss_legendre16(double* x, double* w) {
  const int n = 16;
  for (int i = 0; i < n; ++i) {
    double z = std::cos(kPi * (i + 0.75) / (n + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (z * p1 - p0) / (z * z - 1.0);
      double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    x[i] = z;
    w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

void basis(const Problem& pb, int P, std::vector<double>& rho, std::vector<double>& C) {
  std::vector<double> jz = bessel::j0_zeros(P);
  C.resize(P);
  if (!(pb.H > 0)) {
    rho = jz;
    for (int p = 0; p < P; ++p) C[p] = 1.0 / (std::sqrt(kPi) * rho[p] * std::fabs(bessel::j1(rho[p])));
    return;
  }
  // Dini roots: g(r) = H J0(r) - r J1(r) is H > 0 at 0 and -j J1(j) at each zero j of
  // J0 (alternating sign), so one root lies in (0, j_1) and one in each (j_{p-1}, j_p)
  rho.resize(P);
  const double H = pb.H;
  auto g = [&](double r) {
    double J0, J1;
    bessel::j0j1(r, &J0, &J1);
    return H * J0 - r * J1;
  };
  for (int p = 0; p < P; ++p) {
    double lo = p ? jz[p - 1] : 0.0, hi = jz[p];
    double glo = g(lo);
    for (int it = 0; it < 200 && hi - lo > 1e-15 * hi; ++it) {
      double mid = 0.5 * (lo + hi);
      double gm = g(mid);
      if ((gm > 0) == (glo > 0)) { lo = mid; glo = gm; } else { hi = mid; }
    }
    rho[p] = 0.5 * (lo + hi);
    // a_H(e, e) = 2 pi C^2 (F(1) + H J0(rho)^2), F(1) = rho^2 (J0^2 + J1^2) / 2 - rho J0 J1
    double J0, J1;
    bessel::j0j1(rho[p], &J0, &J1);
    double F1 = rho[p] * rho[p] * 0.5 * (J0 * J0 + J1 * J1) - rho[p] * J0 * J1;
    C[p] = 1.0 / std::sqrt(2.0 * kPi * (F1 + H * J0 * J0));
  }
}

// A^P (row-major, full) and b for the normalised basis.
void assemble(const Problem& pb, const std::vector<double>& rho, const std::vector<double>& C,
              std::vector<double>& A, std::vector<double>& b, int nthreads) {
  const int P = (int)rho.size();
  const double a = pb.a;
  std::vector<double> j0a(P), j1a(P), j01(P), j11(P);
  for (int p = 0; p < P; ++p) {
    bessel::j0j1(rho[p] * a, &j0a[p], &j1a[p]);
    bessel::j0j1(rho[p], &j01[p], &j11[p]);
  }
  A.assign((size_t)P * P, 0.0);
  // F_ij(r) = rho_i r J0(rho_i r) J0'(rho_j r) = -rho_i r J0(rho_i r) J1(rho_j r)
  parallel_for(P, nthreads, [&](int64_t ii) {
    int i = (int)ii;
    for (int j = 0; j < P; ++j) {
      if (i == j) {
        auto Fd = [&](double r, double J0, double J1) {
          double j0p = -J1;
          return rho[i] * rho[i] * r * r * (0.5 * J0 * J0 + 0.5 * j0p * j0p) + rho[i] * r * J0 * j0p;
        };
        A[(size_t)i * P + i] = 2.0 * kPi * C[i] * C[i] * (Fd(1.0, j01[i], j11[i]) - Fd(a, j0a[i], j1a[i]));
        continue;
      }
      double Fij1 = -rho[i] * j01[i] * j11[j];
      double Fji1 = -rho[j] * j01[j] * j11[i];
      double Fija = -rho[i] * a * j0a[i] * j1a[j];
      double Fjia = -rho[j] * a * j0a[j] * j1a[i];
      A[(size_t)i * P + j] = 2.0 * kPi * C[i] * C[j] * rho[i] * rho[j] / (rho[j] * rho[j] - rho[i] * rho[i]) *
                             ((Fji1 - Fij1) - (Fjia - Fija));
    }
  }, 16);
  if (pb.H > 0) {
    // Robin boundary term of a_H on the unit circle
    for (int i = 0; i < P; ++i)
      for (int j = 0; j < P; ++j) A[(size_t)i * P + j] += 2.0 * kPi * pb.H * C[i] * j01[i] * C[j] * j01[j];
  }
  b.resize(P);
  if (pb.kind == 0) {
    // b_p = -2 pi C_p (J0(rho_p a) - J0(rho_p))
    for (int p = 0; p < P; ++p) b[p] = -2.0 * kPi * C[p] * (j0a[p] - j01[p]);
  } else if (pb.kind == 2) {
    // b_p = 2 pi int_a^1 e_p'(r) H'(r) r dr: the c log part in closed form (as for
    // Laplace), the smooth rest by composite 16-point Gauss-Legendre with panels short
    // against the fastest oscillation of e_p' and H'
    const GenShape& G = *pb.gen;
    for (int p = 0; p < P; ++p) b[p] = -2.0 * kPi * C[p] * (j0a[p] - j01[p]) * G.c;
    double gx[16], gw[16];
    gauss_legendre16(gx, gw);
    const double fmax = rho[P - 1] + G.wmax;
    const int panels = std::max(4, (int)std::ceil((1.0 - a) * fmax / 2.0));
    const double hp = (1.0 - a) / panels;
    std::vector<double> rq((size_t)panels * 16), wq((size_t)panels * 16);
    parallel_for(panels, nthreads, [&](int64_t k) {
      for (int i = 0; i < 16; ++i) {
        double r = a + hp * (k + 0.5 * (gx[i] + 1.0));
        rq[(size_t)k * 16 + i] = r;
        wq[(size_t)k * 16 + i] = 0.5 * hp * gw[i] * r * G.dh_smooth(r);
      }
    }, 16);
    parallel_for(P, nthreads, [&](int64_t p) {
      double acc = 0.0;
      for (size_t q = 0; q < rq.size(); ++q) acc -= wq[q] * rho[p] * bessel::j1(rho[p] * rq[q]);
      b[p] += 2.0 * kPi * C[p] * acc;
    }, 1);
  } else {
    // Green's formula with u = Y0(kp r), v = J0(rho_p r):
    // int_a^1 r u' v' = [r (kp^2 u v' - rho^2 u' v)]_a^1 / (kp^2 - rho^2)
    double kp = pb.kp;
    double y0a, y1a, y01, y11;
    y0a = bessel::y0(kp * a);
    y1a = bessel::y1(kp * a);
    y01 = bessel::y0(kp);
    y11 = bessel::y1(kp);
    for (int p = 0; p < P; ++p) {
      auto g = [&](double r, double u, double up, double v, double vp) {
        return r * (kp * kp * u * vp - rho[p] * rho[p] * up * v);
      };
      double g1 = g(1.0, y01, -kp * y11, j01[p], -rho[p] * j11[p]);
      double ga = g(a, y0a, -kp * y1a, j0a[p], -rho[p] * j1a[p]);
      b[p] = 2.0 * kPi * C[p] * (g1 - ga) / (kp * kp - rho[p] * rho[p]);
      if (pb.H > 0) b[p] += 2.0 * kPi * pb.H * y01 * C[p] * j01[p];
    }
  }
}

int fit_search(const Problem& pb, double kappa, double eps, int force_P, int nthreads, FitResult& out,
               std::string& msg);

}  // namespace

int64_t circle_size(double x, double eta) {
  int64_t M = (int64_t)std::floor(x) + 1;
  if (M % 2) ++M;
  if (!(eta > 0)) return M;
  double leta = std::log(eta / 2.0);
  for (;;) {
    double l1 = bessel::log_abs_jn_tail((double)M, x);
    double l2 = bessel::log_abs_jn_tail(2.0 * M, x);
    if (std::isfinite(l1) && std::isfinite(l2)) {
      double mx = std::max(l1, l2);
      double ls = mx + std::log(std::exp(l1 - mx) + std::exp(l2 - mx));
      if (ls <= leta) return M;
    }
    M += 2;
  }
}

int sbd_fit(int kind, double a, double eps, double kappa, int force_P, int nthreads,
            FitResult& out, std::string& msg) {
  if (!(a > 0 && a < 1) || !(eps > 0)) {
    msg = "need 0 < delta_min < delta_max and eps > 0";
    return -1;
  }
  Problem pb{kind, a, 0.0};
  out = FitResult();
  out.kind = kind;
  if (kind == 1) {
    const double y01 = bessel::y0_zero_at_least(0.0);
    out.kappa = kappa;
    if (kappa > 0 && kappa < y01) {
      // Dini basis (Robin condition), no rescaling
      pb.kp = kappa;
      pb.H = kappa * bessel::y1(kappa) / bessel::y0(kappa);
      out.kappa_p = kappa;
      out.lam = 1.0;
      out.robin_H = pb.H;
    } else {
      double kp = bessel::y0_zero_at_least(kappa);
      pb.kp = kp;
      out.kappa_p = kp;
      out.lam = kappa / kp;
      pb.a = out.lam * a;
    }
  }
  return fit_search(pb, kappa, eps, force_P, nthreads, out, msg);
}

namespace {

// The order search and the circles of a fit set up in pb (kinds 0, 1, 2).
int fit_search(const Problem& pb, double kappa, double eps, int force_P, int nthreads, FitResult& out,
               std::string& msg) {
  const int kind = pb.kind;
  out.a = pb.a;
  const double tol = 0.5 * eps;
  int Plo = (int)std::ceil(1.0 / pb.a);
  if (kind == 1) Plo = std::max(Plo, (int)std::ceil(pb.kp / kPi) + 1);
  if (kind == 2) {
    // the series must reach the kernel's frequency (rho_P >= w delta_max) within the
    // Gram matrix's conditioning range P <~ 6 / a: refuse before assembling a P x P system
    Plo = std::max(Plo, (int)std::ceil(pb.gen->wmax / kPi) + 1);
    if (Plo > (int)std::ceil(6.0 / pb.a)) {
      msg = "general kernel oscillates too fast for the SBD on [delta_min, delta_max] (w delta_min above about 6 pi)";
      return -4;
    }
  }
  const int Pcap = std::max(Plo, (int)std::ceil(6.0 / pb.a));
  // error model from the Section 4.1 remark (decay ~ exp(-3.6 gamma)): start bracket
  double gam = 2.0 + std::log(3.3e-4 / tol) / 3.55;
  int Phi = force_P > 0 ? force_P : std::min(Pcap, std::max(Plo, (int)std::ceil((gam + 0.6) / pb.a)));
  // check grid s_j = a (1/a)^((j/(n-1))^2)
  std::vector<double> s(kNCheck), gs(kNCheck);
  for (int j = 0; j < kNCheck; ++j) {
    double t = (double)j / (kNCheck - 1);
    s[j] = pb.a * std::pow(1.0 / pb.a, t * t);
    gs[j] = target(pb, s[j]);
  }
  for (int attempt = 0; attempt < 8; ++attempt) {
    std::vector<double> rho, C, A, b;
    basis(pb, Phi, rho, C);
    assemble(pb, rho, C, A, b, nthreads);
    if (!cholesky(A, Phi, nthreads)) {
      msg = "Gram matrix numerically indefinite: tolerance below the SBD floor";
      return -4;
    }
    // forward solve y = L^-1 b (prefix-consistent across orders)
    std::vector<double> y(Phi);
    for (int i = 0; i < Phi; ++i) y[i] = (b[i] - dot(&A[(size_t)i * Phi], y.data(), i)) / A[(size_t)i * Phi + i];
    // B[j][p] = C_p J0(rho_p s_j)
    std::vector<double> B((size_t)kNCheck * Phi);
    parallel_for(kNCheck, nthreads, [&](int64_t j) {
      for (int p = 0; p < Phi; ++p) B[(size_t)j * Phi + p] = C[p] * bessel::j0(rho[p] * s[j]);
    }, 16);
    auto solve = [&](int P, std::vector<double>& alpha) {
      // L^T alpha = y by the update form: each step reads one row of L (contiguous)
      alpha.assign(y.begin(), y.begin() + P);
      for (int k = P - 1; k >= 0; --k) {
        const double* Lk = &A[(size_t)k * Phi];
        const double ak = alpha[k] / Lk[k];
        alpha[k] = ak;
        for (int i = 0; i < k; ++i) alpha[i] -= Lk[i] * ak;
      }
    };
    auto error_at = [&](int P) {
      std::vector<double> alpha;
      solve(P, alpha);
      std::vector<double> e(kNCheck);
      parallel_for(kNCheck, nthreads, [&](int64_t j) {
        e[j] = std::fabs(gs[j] - dot(&B[(size_t)j * Phi], alpha.data(), P));
      }, 64);
      return *std::max_element(e.begin(), e.end());
    };
    int P;
    double err;
    if (force_P > 0) {
      P = Phi;
      err = error_at(P);
    } else {
      double ehi = error_at(Phi);
      if (ehi > tol) {
        if (Phi >= Pcap) {
          msg = "tolerance below the reachable SBD floor";
          return -4;
        }
        Phi = std::min(Pcap, (int)std::ceil(Phi * 1.4));
        continue;
      }
      int lo = std::max(Plo, (int)std::floor(Phi * 0.45));
      if (error_at(lo) <= tol) lo = Plo;
      int hi = Phi;
      while (lo < hi) {
        int mid = (lo + hi) / 2;
        if (error_at(mid) <= tol) hi = mid;
        else lo = mid + 1;
      }
      P = lo;
      err = error_at(P);
    }
    out.P = P;
    out.err = err;
    out.rho.assign(rho.begin(), rho.begin() + P);
    out.C.assign(C.begin(), C.begin() + P);
    solve(P, out.alpha);
    out.coef.resize(P);
    out.radii.resize(P);
    out.M.resize(P);
    for (int p = 0; p < P; ++p) {
      out.coef[p] = out.alpha[p] * out.C[p];
      out.radii[p] = out.rho[p] * out.lam;
    }
    if (kind == 2) {
      // the enforced circles K = sum_t mu_t J0(omega_t s) join the fitted ones
      const GenShape& G = *pb.gen;
      out.n_enforced = (int)G.om.size();
      for (size_t t = 0; t < G.om.size(); ++t) {
        out.coef.push_back(G.mu[t]);
        out.radii.push_back(G.om[t]);
        out.M.push_back(0);
      }
      out.P = P + out.n_enforced;
      out.constant = G.clogd + G.H1;
    }
    const int Pt = out.P;
    parallel_for(Pt, nthreads, [&](int64_t p) {
      double eta = eps / (2.0 * Pt * std::fabs(out.coef[p]));
      out.M[p] = circle_size(out.radii[p], eta);
    }, 16);
    if (kind == 1) {
      out.extra_radius = kappa;
      out.extra_M = circle_size(kappa, eps / (2.0 * P));
    }
    return 0;
  }
  msg = "order search did not converge";
  return -4;
}

// n roots of J1 nearest w (ascending); J1 has one zero between consecutive zeros of J0.
std::vector<double> j1_roots_near(double w, int n) {
  const int kmax = (int)(w / kPi) + n + 4;
  std::vector<double> jz = bessel::j0_zeros(kmax + 1), z(kmax);
  for (int k = 0; k < kmax; ++k) {
    double lo = jz[k], hi = jz[k + 1];
    const bool slo = bessel::j1(lo) > 0;
    for (int it = 0; it < 200 && hi - lo > 1e-15 * hi; ++it) {
      double mid = 0.5 * (lo + hi);
      if ((bessel::j1(mid) > 0) == slo) lo = mid; else hi = mid;
    }
    z[k] = 0.5 * (lo + hi);
  }
  std::stable_sort(z.begin(), z.end(), [&](double x, double y) { return std::fabs(x - w) < std::fabs(y - w); });
  z.resize(n);
  std::sort(z.begin(), z.end());
  return z;
}

}  // namespace

double general_eval(const GeneralKernel& g, double r) {
  double v = g.c_log != 0.0 ? g.c_log * std::log(r) : 0.0;
  for (const TrigTerm& t : g.terms) v += std::pow(r, t.m) * (t.a * std::sin(t.w * r) + t.b * std::cos(t.w * r));
  return v;
}

int sbd_fit_general(const GeneralKernel& gk, double delta_max, double a, double eps, int nthreads,
                    FitResult& out, std::string& msg) {
  if (!(a > 0 && a < 1) || !(eps > 0) || !(delta_max > 0)) {
    msg = "need 0 < delta_min < delta_max and eps > 0";
    return -1;
  }
  GenShape G;
  G.c = gk.c_log;
  G.clogd = gk.c_log * std::log(delta_max);
  for (const TrigTerm& t : gk.terms) {
    // r^m (a sin(w r) + b cos(w r)) at r = delta_max s
    const double W = t.w * delta_max, sc = std::pow(delta_max, t.m);
    if (t.a != 0.0 && W != 0.0) G.T[TrigKey{t.m, W, 1}] += t.a * sc;
    if (t.b != 0.0) G.T[TrigKey{t.m, W, 0}] += t.b * sc;
    G.wmax = std::max(G.wmax, W);
  }
  G.dT = trig_d(G.T, 0.0);
  const int n = gk.enforce;
  if (n > 0) {
    // lambda_s = (-Delta)^s g at s = 1, s = 1..n+1 (c log s is harmonic)
    std::vector<double> lam;
    TrigMap f = G.T;
    for (int s = 0; s <= n; ++s) {
      f = trig_neg_lap(f);
      lam.push_back(trig_eval(f, 1.0));
    }
    double mean = 0.0;
    for (int s = 0; s < n; ++s) mean += lam[s + 1] / lam[s];
    mean /= n;
    if (!std::isfinite(mean) || mean == 0.0) {
      msg = "multi-Dirichlet enforcement needs nonzero Laplacian iterates of G at r = delta_max";
      return -1;
    }
    G.om = j1_roots_near(std::sqrt(std::fabs(mean)), n);
    // sum_t mu_t omega_t^(2s) J0(omega_t) = lambda_s, s = 1..n (Gaussian elimination, partial pivoting)
    std::vector<double> M((size_t)n * n), rhs(lam.begin(), lam.begin() + n);
    for (int s = 0; s < n; ++s)
      for (int t = 0; t < n; ++t) M[(size_t)s * n + t] = std::pow(G.om[t], 2.0 * (s + 1)) * bessel::j0(G.om[t]);
    for (int c = 0; c < n; ++c) {
      int pr = c;
      for (int r = c + 1; r < n; ++r)
        if (std::fabs(M[(size_t)r * n + c]) > std::fabs(M[(size_t)pr * n + c])) pr = r;
      for (int t = 0; t < n; ++t) std::swap(M[(size_t)c * n + t], M[(size_t)pr * n + t]);
      std::swap(rhs[c], rhs[pr]);
      for (int r = c + 1; r < n; ++r) {
        double l = M[(size_t)r * n + c] / M[(size_t)c * n + c];
        for (int t = c; t < n; ++t) M[(size_t)r * n + t] -= l * M[(size_t)c * n + t];
        rhs[r] -= l * rhs[c];
      }
    }
    G.mu.assign(n, 0.0);
    for (int c = n - 1; c >= 0; --c) {
      double v = rhs[c];
      for (int t = c + 1; t < n; ++t) v -= M[(size_t)c * n + t] * G.mu[t];
      G.mu[c] = v / M[(size_t)c * n + c];
    }
    for (double w : G.om) G.wmax = std::max(G.wmax, w);
  }
  G.H1 = G.h(1.0);
  Problem pb{2, a, 0.0};
  pb.gen = &G;
  out = FitResult();
  out.kind = 2;
  return fit_search(pb, 0.0, eps, 0, nthreads, out, msg);
}

std::complex<double> g_sbd(const FitResult& fit, int kind, double delta_max, double wavenumber, double r) {
  double s = r / delta_max;
  double series = 0.0;
  for (int p = 0; p < fit.P; ++p) series += fit.coef[p] * bessel::j0(fit.radii[p] * s);
  if (kind == 0) return {-(std::log(delta_max) + series) / (2.0 * kPi), 0.0};
  if (kind == 2) return {fit.constant + series, 0.0};
  return {-0.25 * series, 0.25 * bessel::j0(wavenumber * r)};
}

NearTables near_tables(const FitResult& fit, int kind, double delta_max, double U, double wavenumber,
                       int deg, const GeneralKernel* gk) {
  NearTables t;
  t.deg = deg;
  t.U = U;
  const int n = deg + 1;
  std::vector<double> fa(n), fb(n);
  // the samples are independent (each sums the P-term series): spread over host threads
  const int nth = (int)std::min<unsigned>(16, std::max(1u, std::thread::hardware_concurrency()));
  parallel_for(n, nth, [&](int64_t jj) {
    const int j = (int)jj;
    double th = kPi * (j + 0.5) / n;
    double u = 0.5 * U * (1.0 + std::cos(th));
    double r = std::sqrt(u);
    if (kind == 2) {
      // Chebyshev nodes in r: D = (c_log / 2) log u + (G - c_log log r) - G_SBD(r)
      r = 0.5 * std::sqrt(U) * (1.0 + std::cos(th));
      u = r * r;
    }
    std::complex<double> gs = g_sbd(fit, kind, delta_max, wavenumber, r);
    if (kind == 2) {
      GeneralKernel trig = *gk;
      trig.c_log = 0.0;
      fa[j] = 0.5 * gk->c_log;
      fb[j] = general_eval(trig, r) - gs.real();
    } else if (kind == 0) {
      // D = -(1/4 pi) log u - G_SBD(r)
      fa[j] = -1.0 / (4.0 * kPi);
      fb[j] = -gs.real();
    } else {
      // D = (i/4) H0(kr) - G_SBD = -(1/4)(Y0(kr) - Y0_SBD); Y0(kr) = (1/pi) J0(kr) log u + smooth
      double kr = wavenumber * r;
      double J0 = bessel::j0(kr);
      double Y0 = bessel::y0(kr);
      fa[j] = -0.25 * J0 / kPi;
      fb[j] = -0.25 * (Y0 - J0 * std::log(u) / kPi) - gs.real();
    }
  }, 1);
  auto cheb = [&](const std::vector<double>& f) {
    std::vector<double> c(n);
    for (int k = 0; k < n; ++k) {
      double acc = 0;
      for (int j = 0; j < n; ++j) acc += f[j] * std::cos(kPi * k * (j + 0.5) / n);
      c[k] = (k == 0 ? 1.0 : 2.0) * acc / n;
    }
    return c;
  };
  t.A = cheb(fa);
  t.B = cheb(fb);
  t.self = -g_sbd(fit, kind, delta_max, wavenumber, 0.0);
  return t;
}

double es_hat(double beta, double alpha, double t) {
  // int_{-alpha}^{alpha} exp(beta (sqrt(1 - (x/alpha)^2) - 1)) cos(t x) dx by Gauss-Legendre
  // on the substitution x = alpha sin(theta), which removes the square-root endpoint behaviour.
  const int n = 200;
  double acc = 0.0;
  // composite midpoint rule in theta on [-pi/2, pi/2] is spectrally accurate for this smooth periodic-like integrand
  for (int i = 0; i < n; ++i) {
    double th = -0.5 * kPi + kPi * (i + 0.5) / n;
    double x = alpha * std::sin(th);
    double w = alpha * std::cos(th) * (kPi / n);
    acc += w * std::exp(beta * (std::cos(th) - 1.0)) * std::cos(t * x);
  }
  return acc;
}

std::vector<double> es_hat_cheb(double beta, double alpha, double tmax, int deg) {
  const int n = deg + 1;
  std::vector<double> f(n), c(n);
  for (int j = 0; j < n; ++j) {
    double th = kPi * (j + 0.5) / n;
    double t = 0.5 * tmax * (1.0 + std::cos(th));
    f[j] = es_hat(beta, alpha, t);
  }
  for (int k = 0; k < n; ++k) {
    double acc = 0;
    for (int j = 0; j < n; ++j) acc += f[j] * std::cos(kPi * k * (j + 0.5) / n);
    c[k] = (k == 0 ? 1.0 : 2.0) * acc / n;
  }
  return c;
}

}  // namespace sbd
