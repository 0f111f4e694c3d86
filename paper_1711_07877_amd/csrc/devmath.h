// Small device helpers shared by the plan kernels: the exact pair predicate, Chebyshev
// evaluation and the exponential-of-semicircle (ES) spreading kernel.
#pragma once
#include <hip/hip_runtime.h>

namespace sbd {

__device__ __forceinline__ double d2_exact(double ax, double ay, double bx, double by) {
  // (ax-bx)*(ax-bx) + (ay-by)*(ay-by) with round-to-nearest and no fused multiply-add
  double dx = __dsub_rn(ax, bx);
  double dy = __dsub_rn(ay, by);
  return __dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy));
}

// sum_k c[k] T_k(t), t in [-1, 1] (Clenshaw)
__device__ __forceinline__ double cheb_eval(const double* c, int deg, double t) {
  double b1 = 0.0, b2 = 0.0;
  for (int k = deg; k >= 1; --k) {
    double tmp = 2.0 * t * b1 - b2 + c[k];
    b2 = b1;
    b1 = tmp;
  }
  return t * b1 - b2 + c[0];
}

// exp(beta (sqrt(1 - x^2) - 1)) at x = d * two_over_w, zero for |x| >= 1
template <typename T>
__device__ __forceinline__ T es_kernel(T d, T two_over_w, T beta) {
  T x = d * two_over_w;
  T y = T(1) - x * x;
  return y > T(0) ? exp(beta * (sqrt(y) - T(1))) : T(0);
}

// FP32: the hardware square root and base-2 exponential (about 1 ulp each); with
// |beta (sqrt(y) - 1)| <= beta the relative error of a weight stays near 1e-6,
// far below the kernel's own approximation error at the FP32 path's tolerances.
template <>
__device__ __forceinline__ float es_kernel<float>(float d, float two_over_w, float beta) {
  const float x = d * two_over_w;
  const float y = 1.0f - x * x;
  return y > 0.0f ? __builtin_amdgcn_exp2f(beta * 1.4426950408889634f * (__builtin_amdgcn_sqrtf(y) - 1.0f)) : 0.0f;
}

}  // namespace sbd
