// Host FP64 Bessel functions of integer order used by the off-line fit.
//
// Methods (all published, written from their definitions):
//  * x <= kSmallArg: Miller's backward recurrence for J_n, normalised with
//    J_0 + 2 sum_k J_2k = 1 (DLMF 10.74(iv), 10.12.4); Y0 and Y1 from the
//    Neumann expansions Y0 = (2/pi)(ln(x/2)+g) J0 - (4/pi) sum (-1)^k J_2k / k
//    and its derivative (DLMF 10.23(ii)).
//  * x > kSmallArg: Hankel asymptotic expansions (DLMF 10.17.3, 10.17.4).
//  * |J_n(x)| for n > x in the circle-size rule: Debye's expansion
//    (DLMF 10.19.3 with 10.41.10) away from the turning point.
//  * Zeros of J0 and Y0: McMahon's expansion (DLMF 10.21(vi)) refined by
//    Newton steps with J0' = -J1, Y0' = -Y1.
#pragma once
#include <vector>

namespace sbd {
namespace bessel {

constexpr double kSmallArg = 25.0;

double j0(double x);
double j1(double x);
double y0(double x);
double y1(double x);
void   j0j1(double x, double* j0, double* j1);
// J_n(x) for integer n >= 0 and x >= 0 (backward recurrence; used for small x).
double jn_small(int n, double x);
// log |J_nu(x)| upper estimate for nu > x > 0 (Debye); returns +inf near the turning point.
double log_abs_jn_tail(double nu, double x);
// First n positive zeros of J0 / Y0.
std::vector<double> j0_zeros(int n);
std::vector<double> y0_zeros(int n);
// Smallest zero of Y0 that is >= x.
double y0_zero_at_least(double x);

}  // namespace bessel
}  // namespace sbd
