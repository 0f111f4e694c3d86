// Kernel templates of the compiled whole-column convolution (included by the instance
// sources; see colconv.hip for the method).
#pragma once
#include <hip/hip_runtime.h>

#include "colconv.h"
#include "dft.h"

namespace sbd {
namespace cc {

using dft::Dft;

template <int PAD>
__device__ __forceinline__ int lidx(int e) { return e + e / PAD; }

template <typename T, int R0, int R1, int R2, int R3>
struct CcShape {
  static constexpr int L = R0 * R1 * R2 * R3;
  static constexpr int PAD = R0;
  static constexpr int LDS_ELEMS = L + L / PAD + 1;
  // twiddle tables, entries [k][r - 1] of W_{Ns R}^{r k}, k < Ns, stages back to back:
  // forward stages 1..3, then inverse stages 1..3 (stage 0 of each needs none)
  static constexpr int F1 = 0;
  static constexpr int F2 = F1 + R0 * (R1 - 1);
  static constexpr int F3 = F2 + R0 * R1 * (R2 - 1);
  static constexpr int I1 = F3 + R0 * R1 * R2 * (R3 - 1);
  static constexpr int I2 = I1 + R3 * (R2 - 1);
  static constexpr int I3 = I2 + R3 * R2 * (R1 - 1);
  static constexpr int TW = I3 + R3 * R2 * R1 * (R0 - 1);
};


// Generic LDS stage (radix R, Ns = NS, direction DIR) over the padded column buffer.
template <typename T, int NT, int L, int PAD, int R, int NS, int DIR>
__device__ __forceinline__ void cc_stage(cplx<T>* __restrict__ buf, const cplx<T>* __restrict__ tw) {
  constexpr int LR = L / R;
  constexpr int NB = (LR + NT - 1) / NT;
  const int t = threadIdx.x;
  cplx<T> v[NB][R];
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const int j = t + i * NT;
    if (LR % NT == 0 || j < LR) {
      cplx<T> w[R];
      if constexpr (NS > 1) {
        const int k = j % NS;
#pragma unroll
        for (int r = 1; r < R; ++r) w[r] = tw[k * (R - 1) + (r - 1)];
      }
      if constexpr (LR % PAD == 0) {
        const int base = lidx<PAD>(j);
#pragma unroll
        for (int r = 0; r < R; ++r) v[i][r] = buf[base + r * (LR + LR / PAD)];
      } else {
#pragma unroll
        for (int r = 0; r < R; ++r) v[i][r] = buf[lidx<PAD>(j + r * LR)];
      }
      if constexpr (NS > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) v[i][r] = cmul<T>(v[i][r], w[r]);
      }
      Dft<T, R>::run(v[i], DIR);
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const int j = t + i * NT;
    if (LR % NT == 0 || j < LR) {
      const int g = j / NS, k = j - g * NS;
      const int dst = g * NS * R + k;
      if constexpr (NS % PAD == 0) {
        const int base = lidx<PAD>(dst);
#pragma unroll
        for (int r = 0; r < R; ++r) buf[base + r * (NS + NS / PAD)] = v[i][r];
      } else {
#pragma unroll
        for (int r = 0; r < R; ++r) buf[lidx<PAD>(dst + r * NS)] = v[i][r];
      }
    }
  }
  __syncthreads();
}

// Offset of the second of two column buffers of LE elements each (of EB bytes): LE rounded
// up so that the buffers sit half the 64 four-byte LDS banks apart.
template <int EB>
constexpr int cc_second_buffer(int le) {
  constexpr int per = 256 / EB, half = 128 / EB;  // elements per 64 banks, per 32 banks
  return ((le - half + per - 1) / per) * per + half;
}

// The same stage over two buffers (BOFF elements apart) by the same threads: one set of
// twiddles serves both.
template <typename T, int NT, int L, int PAD, int BOFF, int R, int NS, int DIR>
__device__ __forceinline__ void cc_stage2(cplx<T>* __restrict__ buf, const cplx<T>* __restrict__ tw) {
  constexpr int LR = L / R;
  constexpr int NB = (LR + NT - 1) / NT;
  const int t = threadIdx.x;
  cplx<T> v[NB][2][R];
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const int j = t + i * NT;
    if (LR % NT == 0 || j < LR) {
      cplx<T> w[R];
      if constexpr (NS > 1) {
        const int k = j % NS;
#pragma unroll
        for (int r = 1; r < R; ++r) w[r] = tw[k * (R - 1) + (r - 1)];
      }
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        const cplx<T>* b = buf + c * BOFF;
        if constexpr (LR % PAD == 0) {
          const int base = lidx<PAD>(j);
#pragma unroll
          for (int r = 0; r < R; ++r) v[i][c][r] = b[base + r * (LR + LR / PAD)];
        } else {
#pragma unroll
          for (int r = 0; r < R; ++r) v[i][c][r] = b[lidx<PAD>(j + r * LR)];
        }
        if constexpr (NS > 1) {
#pragma unroll
          for (int r = 1; r < R; ++r) v[i][c][r] = cmul<T>(v[i][c][r], w[r]);
        }
        Dft<T, R>::run(v[i][c], DIR);
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const int j = t + i * NT;
    if (LR % NT == 0 || j < LR) {
      const int g = j / NS, k = j - g * NS;
      const int dst = g * NS * R + k;
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        cplx<T>* b = buf + c * BOFF;
        if constexpr (NS % PAD == 0) {
          const int base = lidx<PAD>(dst);
#pragma unroll
          for (int r = 0; r < R; ++r) b[base + r * (NS + NS / PAD)] = v[i][c][r];
        } else {
#pragma unroll
          for (int r = 0; r < R; ++r) b[lidx<PAD>(dst + r * NS)] = v[i][c][r];
        }
      }
    }
  }
  __syncthreads();
}

template <typename T, bool CH, int NT, int MINB, int R0, int R1, int R2, int R3>
__global__ void __launch_bounds__(NT, MINB) k_colconv(CcArgs a) {
  using S = CcShape<T, R0, R1, R2, R3>;
  constexpr int L = S::L, PAD = S::PAD;
  extern __shared__ unsigned char smem_raw[];
  cplx<T>* buf = reinterpret_cast<cplx<T>*>(smem_raw);
  const cplx<T>* __restrict__ tw = reinterpret_cast<const cplx<T>*>(a.tw);
  // consecutive columns on one XCD (blocks are dispatched round-robin over the 8 XCDs)
  const int64_t nb = (int64_t)gridDim.x;
  int64_t bx = blockIdx.x;
  {
    const int64_t q = nb >> 3, rem = nb & 7, x = bx & 7;
    bx = x * q + (x < rem ? x : rem) + (bx >> 3);
  }
  const int64_t col = bx;
  cplx<T>* __restrict__ g = reinterpret_cast<cplx<T>*>(a.data) + blockIdx.y * a.sbatch;
  const int t = threadIdx.x;
  const int64_t pitch = a.pitch;
  // element (row e, this column): natural rows, or rows interleaved in pairs (the two rows
  // of a pair side by side per column, as the paired real-row transforms store them)
  const bool ilv = a.ilv == 2;
  auto off = [&](int e) -> int64_t {
    return ilv ? ((((int64_t)(e >> 1) * pitch + col) << 1) | (int64_t)(e & 1)) : (int64_t)e * pitch + col;
  };

  // forward stage 0 (R0, Ns = 1): inputs j + r L/R0 from global memory, r < R0/2 (the
  // rest lie beyond n_in <= L/2 and are zero), outputs to R0 j + r
  {
    constexpr int R = R0, LR = L / R0, NB = (LR + NT - 1) / NT;
    cplx<T> v[NB][R];
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int j = t + i * NT;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        v[i][r] = mk<T>(T(0), T(0));
        if (r < R / 2 && (LR % NT == 0 || j < LR) && j + r * LR < a.n_in) v[i][r] = g[off(j + r * LR)];
      }
    }
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int j = t + i * NT;
      if (LR % NT == 0 || j < LR) {
#pragma unroll
        for (int r = R / 2; r < R; ++r) v[i][r] = mk<T>(T(0), T(0));
        Dft<T, R>::run(v[i], -1);
#pragma unroll
        for (int r = 0; r < R; ++r) buf[lidx<PAD>(R * j + r)] = v[i][r];
      }
    }
    __syncthreads();
  }
  cc_stage<T, NT, L, PAD, R1, R0, -1>(buf, tw + S::F1);
  cc_stage<T, NT, L, PAD, R2, R0 * R1, -1>(buf, tw + S::F2);
  // forward stage 3 (R3, Ns = L/R3), symbol, inverse stage 0 (R3, Ns = 1)
  {
    constexpr int R = R3, LR = L / R3, NB = (LR + NT - 1) / NT;
    const cplx<T>* __restrict__ tw3 = tw + S::F3;
    const int64_t scol = 2 * col <= a.mx ? col : a.mx - col;
    const T* __restrict__ hr = reinterpret_cast<const T*>(a.sym) + scol * (int64_t)(L / 2 + 1) * (CH ? 2 : 1);
    cplx<T> v[NB][R];
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int j = t + i * NT;
      if (LR % NT == 0 || j < LR) {
        cplx<T> w[R];
#pragma unroll
        for (int r = 1; r < R; ++r) w[r] = tw3[j * (R - 1) + (r - 1)];
        T h[R], hi[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const int e = j + r * LR;
          const int m = e <= L / 2 ? e : L - e;
          if constexpr (CH) {
            const cplx<T> hv = reinterpret_cast<const cplx<T>*>(hr)[m];
            h[r] = hv.x;
            hi[r] = hv.y;
          } else {
            h[r] = hr[m];
            hi[r] = T(0);
          }
        }
        if constexpr (LR % PAD == 0) {
          const int base = lidx<PAD>(j);
#pragma unroll
          for (int r = 0; r < R; ++r) v[i][r] = buf[base + r * (LR + LR / PAD)];
        } else {
#pragma unroll
          for (int r = 0; r < R; ++r) v[i][r] = buf[lidx<PAD>(j + r * LR)];
        }
#pragma unroll
        for (int r = 1; r < R; ++r) v[i][r] = cmul<T>(v[i][r], w[r]);
        Dft<T, R>::run(v[i], -1);
#pragma unroll
        for (int r = 0; r < R; ++r) {
          if constexpr (CH) v[i][r] = cmul<T>(v[i][r], mk<T>(h[r], hi[r]));
          else v[i][r] = cscale<T>(v[i][r], h[r]);
        }
        Dft<T, R>::run(v[i], +1);
      }
    }
    __syncthreads();
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
  cc_stage<T, NT, L, PAD, R2, R3, +1>(buf, tw + S::I1);
  cc_stage<T, NT, L, PAD, R1, R3 * R2, +1>(buf, tw + S::I2);
  // inverse stage 3 (R0, Ns = L/R0): outputs j + r L/R0 for r < R0/2 to global memory
  {
    constexpr int R = R0, LR = L / R0, NB = (LR + NT - 1) / NT;
    const cplx<T>* __restrict__ tw3 = tw + S::I3;
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int j = t + i * NT;
      if (LR % NT == 0 || j < LR) {
        cplx<T> v[R], w[R];
#pragma unroll
        for (int r = 1; r < R; ++r) w[r] = tw3[j * (R - 1) + (r - 1)];
        if constexpr (LR % PAD == 0) {
          const int base = lidx<PAD>(j);
#pragma unroll
          for (int r = 0; r < R; ++r) v[r] = buf[base + r * (LR + LR / PAD)];
        } else {
#pragma unroll
          for (int r = 0; r < R; ++r) v[r] = buf[lidx<PAD>(j + r * LR)];
        }
#pragma unroll
        for (int r = 1; r < R; ++r) v[r] = cmul<T>(v[r], w[r]);
        Dft<T, R>::run(v, +1);
#pragma unroll
        for (int r = 0; r < R / 2; ++r)
          if (j + r * LR < a.n_out) g[off(j + r * LR)] = v[r];
      }
    }
  }
}

// Threads per column: about a third of the largest stage's butterflies, a power of two in
// [64, 512]; workgroups per CU the compiler may plan registers for: as many as the LDS
// admits, at most four waves per SIMD.
constexpr int cc_pow2_ceil(int x) { int p = 1; while (p < x) p *= 2; return p; }
constexpr int cc_max4(int a, int b, int c, int d) { return (a > b ? a : b) > (c > d ? c : d) ? (a > b ? a : b) : (c > d ? c : d); }
constexpr int cc_min4(int a, int b, int c, int d) { return a < b ? (a < c ? (a < d ? a : d) : (c < d ? c : d)) : (b < c ? (b < d ? b : d) : (c < d ? c : d)); }
template <int R0, int R1, int R2, int R3>
constexpr int cc_threads() {
  constexpr int L = R0 * R1 * R2 * R3;
  constexpr int t = cc_pow2_ceil((L / cc_min4(R0, R1, R2, R3) + 2) / 3);
  return t < 64 ? 64 : (t > 512 ? 512 : t);
}

template <typename T, bool CH, int R0, int R1, int R2, int R3>
int launch_inst(const CcArgs& a, int64_t nbatch, hipStream_t st) {
  using S = CcShape<T, R0, R1, R2, R3>;
  constexpr int NT = cc_threads<R0, R1, R2, R3>();
  constexpr size_t lds = (size_t)S::LDS_ELEMS * sizeof(cplx<T>);
  constexpr int by_lds = (int)((160 * 1024) / lds);
  constexpr int by_waves = 1024 / NT;
  constexpr int MINB = by_lds < 1 ? 1 : (by_lds < by_waves ? by_lds : by_waves);
  auto kfn = k_colconv<T, CH, NT, MINB, R0, R1, R2, R3>;
  if (lds > 65536) (void)hipFuncSetAttribute((const void*)kfn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  hipLaunchKernelGGL(kfn, dim3((unsigned)a.ncols, (unsigned)nbatch), dim3(NT), lds, st, a);
  return hipGetLastError() == hipSuccess ? 0 : -5;
}

}  // namespace cc
}  // namespace sbd
