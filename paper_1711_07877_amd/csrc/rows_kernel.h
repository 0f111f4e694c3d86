// Kernel templates of the compiled real-row transforms (included by the instance
// sources; see rows.hip for the method).
#pragma once
#include <hip/hip_runtime.h>

#include "colconv_kernel.h"
#include "gridrow.h"
#include "rows.h"

namespace sbd {
namespace rr {

using cc::cc_stage;
using cc::lidx;
using dft::Dft;

// Forward: stage 0 (R0, Ns = 1) gathers its inputs z[j + r N/R0], r < R0/2, from the tile
// subgrids (z is zero beyond nx/2 <= N/2), stages 1..3 in LDS leave Z in natural order,
// then X[k] = E[k] + W_M^k O[k] with E, O the even / odd parts of Z.
template <typename T, int NT, int MINB, int R0, int R1, int R2, int R3>
__global__ void __launch_bounds__(NT, MINB) k_r2c(RowArgs k) {
  using S = cc::CcShape<T, R0, R1, R2, R3>;
  constexpr int N = S::L, PAD = R0;
  extern __shared__ unsigned char smem_raw[];
  cplx<T>* buf = reinterpret_cast<cplx<T>*>(smem_raw);
  const RealRowArgs& a = k.a;
  const cplx<T>* __restrict__ tw = reinterpret_cast<const cplx<T>*>(k.tw);
  int64_t Y = blockIdx.x;
  if (a.pair) {
    // spectra interleaved in row pairs (element (Y, k) at ((Y / 2) gpitch + k) 2 + Y % 2):
    // blocks 16 g + w, w < 16, take rows 16 g + 2 (w mod 8) + w / 8, so the two rows of a
    // pair run on one XCD (blocks go round-robin over the 8), eight blocks apart, and their
    // half-filled lines meet in that XCD's L2
    const int64_t g = Y >> 4, w = Y & 15;
    Y = (g << 4) | ((w & 7) << 1) | (w >> 3);
    if (Y >= a.ny) return;
  }
  const int64_t rb = blockIdx.y;
  const int t = threadIdx.x;
  const cplx<T>* sub2 = reinterpret_cast<const cplx<T>*>(a.sub);
  const int tyhi = (int)(Y >> a.log2T);
  int64_t row0 = -1, row1 = -1;
  int ly0 = 0, ly1 = 0;
  if (tyhi < a.nty) { ly0 = (int)(Y - ((int64_t)tyhi << a.log2T)); if (ly0 < a.SG) row0 = rb * a.ntiles + (int64_t)tyhi * a.ntx; }
  if (tyhi >= 1 && tyhi - 1 < a.nty) {
    ly1 = (int)(Y - ((int64_t)(tyhi - 1) << a.log2T));
    if (ly1 < a.SG) row1 = rb * a.ntiles + (int64_t)(tyhi - 1) * a.ntx;
  }
  {
    constexpr int R = R0, LR = N / R0, NB = (LR + NT - 1) / NT;
    cplx<T> v[NB][R];
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int j = t + i * NT;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        v[i][r] = mk<T>(T(0), T(0));
        if (r < R / 2 && (LR % NT == 0 || j < LR)) v[i][r] = gather_pair<T>(sub2, a, 2 * (j + r * LR), ly0, ly1, row0, row1);
      }
    }
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int j = t + i * NT;
      if (LR % NT == 0 || j < LR) {
        Dft<T, R>::run(v[i], -1);
#pragma unroll
        for (int r = 0; r < R; ++r) buf[lidx<PAD>(R * j + r)] = v[i][r];
      }
    }
    __syncthreads();
  }
  cc_stage<T, NT, N, PAD, R1, R0, -1>(buf, tw + S::F1);
  cc_stage<T, NT, N, PAD, R2, R0 * R1, -1>(buf, tw + S::F2);
  cc_stage<T, NT, N, PAD, R3, R0 * R1 * R2, -1>(buf, tw + S::F3);
  const cplx<T>* __restrict__ twM = reinterpret_cast<const cplx<T>*>(k.twM);
  cplx<T>* out = reinterpret_cast<cplx<T>*>(k.grid) + rb * a.sbatch;
  int64_t ostride = 1;
  if (a.pair) {
    out += (Y & ~(int64_t)1) * a.gpitch + (Y & 1);
    ostride = 2;
  } else {
    out += Y * a.gpitch;
  }
  for (int q = t; q <= N; q += NT) {
    const cplx<T> zk = buf[lidx<PAD>(q == N ? 0 : q)];
    cplx<T> zc = buf[lidx<PAD>(q == 0 ? 0 : N - q)];
    zc.y = -zc.y;  // conj(Z[N - k])
    const cplx<T> E = mk<T>(T(0.5) * (zk.x + zc.x), T(0.5) * (zk.y + zc.y));
    const cplx<T> D = mk<T>(T(0.5) * (zk.x - zc.x), T(0.5) * (zk.y - zc.y));
    const cplx<T> O = mk<T>(D.y, -D.x);  // (Z[k] - conj(Z[N - k])) / (2i)
    out[q * ostride] = cadd<T>(E, cmul<T>(twM[q], O));
  }
}

// Inverse: stage 0 (R3, Ns = 1) forms z'[k] = A + i B, A = X[k] + conj(X[N-k]),
// B = (X[k] - conj(X[N-k])) W_M^-k, straight from the row; stages (R2, R1) in LDS; the
// last stage (R0, Ns = N/R0) keeps outputs k + r N/R0 with r < R0/2 (k < nx/2 <= N/2) and
// writes them as real pairs over the row.
template <typename T, int NT, int MINB, int R0, int R1, int R2, int R3>
__global__ void __launch_bounds__(NT, MINB) k_c2r(RowArgs k) {
  using S = cc::CcShape<T, R0, R1, R2, R3>;
  constexpr int N = S::L, PAD = R3;
  extern __shared__ unsigned char smem_raw[];
  cplx<T>* buf = reinterpret_cast<cplx<T>*>(smem_raw);
  const RealRowArgs& a = k.a;
  const cplx<T>* __restrict__ tw = reinterpret_cast<const cplx<T>*>(k.tw);
  const cplx<T>* __restrict__ twM = reinterpret_cast<const cplx<T>*>(k.twM);
  const int64_t Y = blockIdx.x;
  const int64_t rb = blockIdx.y;
  const int t = threadIdx.x;
  cplx<T>* row = reinterpret_cast<cplx<T>*>(k.grid) + rb * a.sbatch + Y * a.gpitch;
  {
    constexpr int R = R3, LR = N / R3, NB = (LR + NT - 1) / NT;
    cplx<T> v[NB][R];
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int j = t + i * NT;
      if (LR % NT == 0 || j < LR) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const int q = j + r * LR;
          const cplx<T> xk = row[q];
          cplx<T> xc = row[N - q];
          xc.y = -xc.y;  // conj(X[N - k])
          const cplx<T> A = cadd<T>(xk, xc);
          cplx<T> w = twM[q];
          w.y = -w.y;  // W_M^{-k}
          const cplx<T> B = cmul<T>(csub<T>(xk, xc), w);
          v[i][r] = mk<T>(A.x - B.y, A.y + B.x);
        }
        Dft<T, R>::run(v[i], +1);
      }
    }
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int j = t + i * NT;
      if (LR % NT == 0 || j < LR) {
#pragma unroll
        for (int r = 0; r < R; ++r) buf[lidx<PAD>(R * j + r)] = v[i][r];
      }
    }
    __syncthreads();
  }
  cc_stage<T, NT, N, PAD, R2, R3, +1>(buf, tw + S::I1);
  cc_stage<T, NT, N, PAD, R1, R3 * R2, +1>(buf, tw + S::I2);
  {
    constexpr int R = R0, LR = N / R0, NB = (LR + NT - 1) / NT;
    const cplx<T>* __restrict__ tw3 = tw + S::I3;
    T* outr = reinterpret_cast<T*>(row);
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int j = t + i * NT;
      if (LR % NT == 0 || j < LR) {
        cplx<T> v[R], w[R];
#pragma unroll
        for (int r = 1; r < R; ++r) w[r] = tw3[j * (R - 1) + (r - 1)];
#pragma unroll
        for (int r = 0; r < R; ++r) v[r] = buf[lidx<PAD>(j + r * LR)];
#pragma unroll
        for (int r = 1; r < R; ++r) v[r] = cmul<T>(v[r], w[r]);
        Dft<T, R>::run(v, +1);
#pragma unroll
        for (int r = 0; r < R / 2; ++r) {
          const int q = j + r * LR;
          if (2 * q < a.nx) outr[2 * q] = v[r].x;
          if (2 * q + 1 < a.nx) outr[2 * q + 1] = v[r].y;
        }
      }
    }
  }
}

// Inverse of two rows per workgroup, reading the pair-interleaved spectra (see k_r2c), the
// two rows' values at one frequency with one contiguous load, and writing each row's real
// values into its own natural row: the pair's storage is read whole in stage 0, before any
// thread writes it, and no other workgroup touches it.  A row at or beyond ny is not written.
template <typename T, int NT, int MINB, int R0, int R1, int R2, int R3>
__global__ void __launch_bounds__(NT, MINB) k_c2r2(RowArgs k) {
  using S = cc::CcShape<T, R0, R1, R2, R3>;
  constexpr int N = S::L, PAD = R3;
  constexpr int BOFF = cc::cc_second_buffer<(int)sizeof(cplx<T>)>(N + N / PAD + 1);
  extern __shared__ unsigned char smem_raw[];
  cplx<T>* buf = reinterpret_cast<cplx<T>*>(smem_raw);
  const RealRowArgs& a = k.a;
  const cplx<T>* __restrict__ tw = reinterpret_cast<const cplx<T>*>(k.tw);
  const cplx<T>* __restrict__ twM = reinterpret_cast<const cplx<T>*>(k.twM);
  const int64_t Y0 = 2 * (int64_t)blockIdx.x;
  const int64_t rb = blockIdx.y;
  const int t = threadIdx.x;
  cplx<T>* rows = reinterpret_cast<cplx<T>*>(k.grid) + rb * a.sbatch + Y0 * a.gpitch;
  {
    constexpr int R = R3, LR = N / R3, NB = (LR + NT - 1) / NT;
    cplx<T> v[NB][2][R];
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int j = t + i * NT;
      if (LR % NT == 0 || j < LR) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const int q = j + r * LR;
          cplx<T> pk[2], pc[2];
          if constexpr (sizeof(T) == 4) {
            const float4 u = reinterpret_cast<const float4*>(rows)[q];
            const float4 v2 = reinterpret_cast<const float4*>(rows)[N - q];
            pk[0] = mk<T>(u.x, u.y);
            pk[1] = mk<T>(u.z, u.w);
            pc[0] = mk<T>(v2.x, v2.y);
            pc[1] = mk<T>(v2.z, v2.w);
          } else {
            pk[0] = rows[2 * q];
            pk[1] = rows[2 * q + 1];
            pc[0] = rows[2 * (N - q)];
            pc[1] = rows[2 * (N - q) + 1];
          }
          cplx<T> w = twM[q];
          w.y = -w.y;  // W_M^{-k}
#pragma unroll
          for (int c = 0; c < 2; ++c) {
            const cplx<T> xk = pk[c];
            const cplx<T> xc = mk<T>(pc[c].x, -pc[c].y);  // conj(X[N - k])
            const cplx<T> A = cadd<T>(xk, xc);
            const cplx<T> B = cmul<T>(csub<T>(xk, xc), w);
            v[i][c][r] = mk<T>(A.x - B.y, A.y + B.x);
          }
        }
#pragma unroll
        for (int c = 0; c < 2; ++c) Dft<T, R>::run(v[i][c], +1);
      }
    }
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int j = t + i * NT;
      if (LR % NT == 0 || j < LR) {
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
          for (int r = 0; r < R; ++r) buf[c * BOFF + lidx<PAD>(R * j + r)] = v[i][c][r];
      }
    }
    __syncthreads();
  }
  cc::cc_stage2<T, NT, N, PAD, BOFF, R2, R3, +1>(buf, tw + S::I1);
  cc::cc_stage2<T, NT, N, PAD, BOFF, R1, R3 * R2, +1>(buf, tw + S::I2);
  {
    constexpr int R = R0, LR = N / R0, NB = (LR + NT - 1) / NT;
    const cplx<T>* __restrict__ tw3 = tw + S::I3;
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int j = t + i * NT;
      if (LR % NT == 0 || j < LR) {
        cplx<T> w[R];
#pragma unroll
        for (int r = 1; r < R; ++r) w[r] = tw3[j * (R - 1) + (r - 1)];
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          if (Y0 + c >= a.ny) continue;
          cplx<T> v[R];
#pragma unroll
          for (int r = 0; r < R; ++r) v[r] = buf[c * BOFF + lidx<PAD>(j + r * LR)];
#pragma unroll
          for (int r = 1; r < R; ++r) v[r] = cmul<T>(v[r], w[r]);
          Dft<T, R>::run(v, +1);
          T* outr = reinterpret_cast<T*>(rows + c * a.gpitch);
#pragma unroll
          for (int r = 0; r < R / 2; ++r) {
            const int q = j + r * LR;
            if (2 * q < a.nx) outr[2 * q] = v[r].x;
            if (2 * q + 1 < a.nx) outr[2 * q + 1] = v[r].y;
          }
        }
      }
    }
  }
}

// Whether an instance has the two-rows-per-workgroup inverse (radices up to 12, both
// buffers in LDS).
template <typename T, int R0, int R1, int R2, int R3>
constexpr bool row_pairs_ok() {
  constexpr int N = R0 * R1 * R2 * R3;
  constexpr int rmax = cc::cc_max4(R0, R1, R2, R3);
  constexpr int le = N + N / (R0 < R3 ? R0 : R3) + 1;
  constexpr int eb = (int)sizeof(cplx<T>);
  return rmax <= 12 && (size_t)(cc::cc_second_buffer<eb>(le) + le) * eb <= 160 * 1024;
}

template <typename T, bool FWD, int R0, int R1, int R2, int R3>
int launch_row(const RowArgs& k, hipStream_t st) {
  using S = cc::CcShape<T, R0, R1, R2, R3>;
  constexpr int NT = cc::cc_threads<R0, R1, R2, R3>();
  constexpr int PADU = FWD ? R0 : R3;  // padding period of the kernel's LDS layout
  if constexpr (row_pairs_ok<T, R0, R1, R2, R3>()) {
    if (k.a.pair && !FWD) {
      constexpr int le = S::L + S::L / PADU + 1;
      constexpr size_t lds = (size_t)(cc::cc_second_buffer<(int)sizeof(cplx<T>)>(le) + le) * sizeof(cplx<T>);
      constexpr int by_lds = (int)((160 * 1024) / lds);
      constexpr int by_waves = 1024 / NT;
      constexpr int MINB = by_lds < 1 ? 1 : (by_lds < by_waves ? by_lds : by_waves);
      auto kfn = k_c2r2<T, NT, MINB, R0, R1, R2, R3>;
      if (lds > 65536) (void)hipFuncSetAttribute((const void*)kfn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      hipLaunchKernelGGL(kfn, dim3((unsigned)((k.a.ny + 1) / 2), (unsigned)k.a.nbatch), dim3(NT), lds, st, k);
      return hipGetLastError() == hipSuccess ? 0 : -5;
    }
  } else {
    if (k.a.pair) return -1;  // no paired inverse for this instance
  }
  constexpr size_t lds = (size_t)(S::L + S::L / PADU + 1) * sizeof(cplx<T>);
  constexpr int by_lds = (int)((160 * 1024) / lds);
  constexpr int by_waves = 1024 / NT;
  constexpr int MINB = by_lds < 1 ? 1 : (by_lds < by_waves ? by_lds : by_waves);
  void (*kfn)(RowArgs) = FWD ? k_r2c<T, NT, MINB, R0, R1, R2, R3> : k_c2r<T, NT, MINB, R0, R1, R2, R3>;
  if (lds > 65536) (void)hipFuncSetAttribute((const void*)kfn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  // paired spectra: whole groups of 16 blocks (the row remap of k_r2c)
  const int64_t nblk = k.a.pair ? (k.a.ny + 15) / 16 * 16 : k.a.ny;
  hipLaunchKernelGGL(kfn, dim3((unsigned)nblk, (unsigned)k.a.nbatch), dim3(NT), lds, st, k);
  return hipGetLastError() == hipSuccess ? 0 : -5;
}

}  // namespace rr
}  // namespace sbd
