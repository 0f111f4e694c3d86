// Grid-row assembly from the per-tile spread subgrids, shared by the real-row transforms.
#pragma once
#include <hip/hip_runtime.h>

#include "common.h"
#include "fft.h"

namespace sbd {

template <typename T>
__device__ __forceinline__ void two_sum_acc(T& s, T& c, T v) {
  T ns = s + v;
  T bb = ns - s;
  c += (s - (ns - bb)) + (v - bb);
  s = ns;
}

template <typename T>
__device__ __forceinline__ cplx<T> gather_pair(const cplx<T>* __restrict__ sub2, const RealRowArgs& a, int X,
                                               int ly0, int ly1, int64_t row0, int64_t row1) {
  // grid cells (Y, X) and (Y, X + 1), X even, as one complex pair: the sum of the
  // (at most 2 x 2) tile subgrids covering them, with a compensated (two-sum)
  // accumulation.  SG and T are even, so a pair never straddles a subgrid row and is
  // read with one load per covering subgrid.  row0/row1 are the subgrid row bases of
  // the two candidate tile rows (negative when absent).
  if (X >= a.nx) return mk<T>(T(0), T(0));
  const int hSG2 = (a.SG * a.SG) >> 1;
  const int tx0 = X >> a.log2T;
  const int lx0 = X - (tx0 << a.log2T);
  const int lx1 = lx0 + (1 << a.log2T);
  const bool c0 = tx0 < a.ntx;
  const bool c1 = tx0 >= 1 && tx0 <= a.ntx && lx1 < a.SG;
  cplx<T> v[4];
  for (int q = 0; q < 4; ++q) v[q] = mk<T>(T(0), T(0));
  if (row0 >= 0) {
    const int64_t b = (row0 + tx0) * hSG2 + ((ly0 * a.SG) >> 1);
    if (c0) v[0] = sub2[b + (lx0 >> 1)];
    if (c1) v[1] = sub2[b - hSG2 + (lx1 >> 1)];
  }
  if (row1 >= 0) {
    const int64_t b = (row1 + tx0) * hSG2 + ((ly1 * a.SG) >> 1);
    if (c0) v[2] = sub2[b + (lx0 >> 1)];
    if (c1) v[3] = sub2[b - hSG2 + (lx1 >> 1)];
  }
  T sx = v[0].x, cx = 0, sy = v[0].y, cy = 0;
  for (int q = 1; q < 4; ++q) {
    two_sum_acc<T>(sx, cx, v[q].x);
    two_sum_acc<T>(sy, cy, v[q].y);
  }
  return mk<T>(sx + cx, sy + cy);
}

}  // namespace sbd
