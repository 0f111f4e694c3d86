// Small DFT butterflies in registers (radices 2, 3, 4, 5, 7, 8, 9, 12, 16) shared by the
// FFT passes: dir = -1 forward (exp(-2 pi i jk/R)), +1 inverse.  Odd radices use
// symmetric sums, 8 = 2 x 4 and the composites 9 = 3 x 3, 12 = 4 x 3, 16 = 4 x 4 are
// Cooley-Tukey inside one thread's registers.
#pragma once
#include <hip/hip_runtime.h>

#include "common.h"

namespace sbd {
namespace dft {

template <typename T> struct K {
  static constexpr T c3 = T(-0.5), s3 = T(0.8660254037844386467637);
  static constexpr T c51 = T(0.3090169943749474241023), s51 = T(0.9510565162951535721164);
  static constexpr T c52 = T(-0.8090169943749474241023), s52 = T(0.5877852522924731291687);
  static constexpr T c71 = T(0.623489801858733530525), s71 = T(0.7818314824680298087084);
  static constexpr T c72 = T(-0.2225209339563144042889), s72 = T(0.9749279121818236070181);
  static constexpr T c73 = T(-0.9009688679024191262361), s73 = T(0.4338837391175581204758);
  static constexpr T r2 = T(0.7071067811865475244008);
};

template <typename T, int R> struct Dft;

template <typename T> struct Dft<T, 2> {
  __device__ static void run(cplx<T>* v, int) {
    cplx<T> a = v[0], b = v[1];
    v[0] = cadd<T>(a, b);
    v[1] = csub<T>(a, b);
  }
};

template <typename T> struct Dft<T, 4> {
  __device__ static void run(cplx<T>* v, int dir) {
    cplx<T> t0 = cadd<T>(v[0], v[2]), t1 = csub<T>(v[0], v[2]);
    cplx<T> t2 = cadd<T>(v[1], v[3]), t3 = cmuli<T>(csub<T>(v[1], v[3]), dir);
    v[0] = cadd<T>(t0, t2);
    v[2] = csub<T>(t0, t2);
    v[1] = cadd<T>(t1, t3);
    v[3] = csub<T>(t1, t3);
  }
};

template <typename T> struct Dft<T, 8> {
  __device__ static void run(cplx<T>* v, int dir) {
    cplx<T> e[4] = {v[0], v[2], v[4], v[6]};
    cplx<T> o[4] = {v[1], v[3], v[5], v[7]};
    Dft<T, 4>::run(e, dir);
    Dft<T, 4>::run(o, dir);
    const T r = K<T>::r2;
    // W8^1 = (1 + dir i)/sqrt2, W8^2 = dir i, W8^3 = (-1 + dir i)/sqrt2
    cplx<T> w1 = mk<T>(r, dir * r), w3 = mk<T>(-r, dir * r);
    cplx<T> o1 = cmul<T>(o[1], w1), o2 = cmuli<T>(o[2], dir), o3 = cmul<T>(o[3], w3);
    v[0] = cadd<T>(e[0], o[0]);
    v[4] = csub<T>(e[0], o[0]);
    v[1] = cadd<T>(e[1], o1);
    v[5] = csub<T>(e[1], o1);
    v[2] = cadd<T>(e[2], o2);
    v[6] = csub<T>(e[2], o2);
    v[3] = cadd<T>(e[3], o3);
    v[7] = csub<T>(e[3], o3);
  }
};

// Odd radix from symmetric sums: u_m = a_m + a_{R-m}, w_m = a_m - a_{R-m},
// y_k = a0 + sum_m u_m cos(2 pi m k/R) + dir i sum_m w_m sin(2 pi m k/R), y_{R-k} likewise with -dir.
template <typename T, int R>
__device__ __forceinline__ void dft_odd(cplx<T>* v, int dir, const T* cs, const T* sn) {
  constexpr int H = (R - 1) / 2;
  cplx<T> u[H], w[H];
  cplx<T> y0 = v[0];
#pragma unroll
  for (int m = 1; m <= H; ++m) {
    u[m - 1] = cadd<T>(v[m], v[R - m]);
    w[m - 1] = csub<T>(v[m], v[R - m]);
    y0 = cadd<T>(y0, u[m - 1]);
  }
  cplx<T> out[R];
  out[0] = y0;
#pragma unroll
  for (int k = 1; k <= H; ++k) {
    cplx<T> re = v[0], im = mk<T>(T(0), T(0));
#pragma unroll
    for (int m = 1; m <= H; ++m) {
      int idx = (m * k) % R;  // cos/sin of 2 pi idx / R
      T c, s;
      if (idx <= H) { c = cs[idx - 1]; s = sn[idx - 1]; }
      else { c = cs[R - idx - 1]; s = -sn[R - idx - 1]; }
      re = mk<T>(re.x + u[m - 1].x * c, re.y + u[m - 1].y * c);
      im = mk<T>(im.x + w[m - 1].x * s, im.y + w[m - 1].y * s);
    }
    cplx<T> di = cmuli<T>(im, dir);
    out[k] = cadd<T>(re, di);
    out[R - k] = csub<T>(re, di);
  }
#pragma unroll
  for (int k = 0; k < R; ++k) v[k] = out[k];
}

template <typename T> struct Dft<T, 3> {
  __device__ static void run(cplx<T>* v, int dir) {
    const T cs[1] = {K<T>::c3}, sn[1] = {K<T>::s3};
    dft_odd<T, 3>(v, dir, cs, sn);
  }
};
template <typename T> struct Dft<T, 5> {
  __device__ static void run(cplx<T>* v, int dir) {
    const T cs[2] = {K<T>::c51, K<T>::c52}, sn[2] = {K<T>::s51, K<T>::s52};
    dft_odd<T, 5>(v, dir, cs, sn);
  }
};
template <typename T> struct Dft<T, 7> {
  __device__ static void run(cplx<T>* v, int dir) {
    const T cs[3] = {K<T>::c71, K<T>::c72, K<T>::c73}, sn[3] = {K<T>::s71, K<T>::s72, K<T>::s73};
    dft_odd<T, 7>(v, dir, cs, sn);
  }
};

// Unit roots cos / sin(2 pi m / N) for the composite radices N in {9, 12, 16}
// (function-local tables, folded to immediates once the butterfly loops are unrolled).
__device__ __forceinline__ double root_cos(int N, int m) {
  constexpr double c9[9] = {1, 0.76604444311897801, 0.17364817766693036, -0.5, -0.93969262078590843,
                            -0.93969262078590843, -0.5, 0.17364817766693036, 0.76604444311897801};
  constexpr double c12[12] = {1, 0.8660254037844386, 0.5, 0, -0.5, -0.8660254037844386,
                              -1, -0.8660254037844386, -0.5, 0, 0.5, 0.8660254037844386};
  constexpr double c16[16] = {1, 0.92387953251128674, 0.70710678118654752, 0.38268343236508977, 0,
                              -0.38268343236508977, -0.70710678118654752, -0.92387953251128674, -1,
                              -0.92387953251128674, -0.70710678118654752, -0.38268343236508977, 0,
                              0.38268343236508977, 0.70710678118654752, 0.92387953251128674};
  return N == 9 ? c9[m] : N == 12 ? c12[m] : c16[m];
}
__device__ __forceinline__ double root_sin(int N, int m) {
  constexpr double s9[9] = {0, 0.64278760968653936, 0.98480775301220802, 0.8660254037844386, 0.34202014332566871,
                            -0.34202014332566871, -0.8660254037844386, -0.98480775301220802, -0.64278760968653936};
  constexpr double s12[12] = {0, 0.5, 0.8660254037844386, 1, 0.8660254037844386, 0.5,
                              0, -0.5, -0.8660254037844386, -1, -0.8660254037844386, -0.5};
  constexpr double s16[16] = {0, 0.38268343236508977, 0.70710678118654752, 0.92387953251128674, 1,
                              0.92387953251128674, 0.70710678118654752, 0.38268343236508977, 0,
                              -0.38268343236508977, -0.70710678118654752, -0.92387953251128674, -1,
                              -0.92387953251128674, -0.70710678118654752, -0.38268343236508977};
  return N == 9 ? s9[m] : N == 12 ? s12[m] : s16[m];
}

// Composite radix N = R1 R2 inside one thread's registers (Cooley-Tukey):
//   X[k1 + R1 k2] = sum_{n2} W_{R2}^{n2 k2} W_N^{n2 k1} sum_{n1} x[R2 n1 + n2] W_{R1}^{n1 k1}.
// Inner twiddles W_N^m with m = N/4, N/2, 3N/4 are applied as exact swaps / negations.
template <typename T, int R1, int R2>
__device__ __forceinline__ void dft_ct(cplx<T>* v, int dir) {
  constexpr int N = R1 * R2;
  cplx<T> a[R2][R1];
#pragma unroll
  for (int n2 = 0; n2 < R2; ++n2) {
#pragma unroll
    for (int n1 = 0; n1 < R1; ++n1) a[n2][n1] = v[R2 * n1 + n2];
    Dft<T, R1>::run(a[n2], dir);
#pragma unroll
    for (int k1 = 1; k1 < R1; ++k1) {
      const int m = (n2 * k1) % N;
      if (m == 0) continue;
      if (4 * m == N) a[n2][k1] = cmuli<T>(a[n2][k1], dir);
      else if (2 * m == N) a[n2][k1] = mk<T>(-a[n2][k1].x, -a[n2][k1].y);
      else if (4 * m == 3 * N) a[n2][k1] = cmuli<T>(a[n2][k1], -dir);
      else {
        const T c = (T)root_cos(N, m), sn = (T)root_sin(N, m);
        a[n2][k1] = cmul<T>(a[n2][k1], mk<T>(c, dir > 0 ? sn : -sn));
      }
    }
  }
#pragma unroll
  for (int k1 = 0; k1 < R1; ++k1) {
    cplx<T> b[R2];
#pragma unroll
    for (int n2 = 0; n2 < R2; ++n2) b[n2] = a[n2][k1];
    Dft<T, R2>::run(b, dir);
#pragma unroll
    for (int k2 = 0; k2 < R2; ++k2) v[k1 + R1 * k2] = b[k2];
  }
}

template <typename T> struct Dft<T, 9> {
  __device__ static void run(cplx<T>* v, int dir) { dft_ct<T, 3, 3>(v, dir); }
};
template <typename T> struct Dft<T, 12> {
  __device__ static void run(cplx<T>* v, int dir) { dft_ct<T, 4, 3>(v, dir); }
};
template <typename T> struct Dft<T, 16> {
  __device__ static void run(cplx<T>* v, int dir) { dft_ct<T, 4, 4>(v, dir); }
};

}  // namespace dft
}  // namespace sbd
