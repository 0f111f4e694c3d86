// Hand-written mixed-radix (2,3,4,5,7,8) Stockham FFT for gfx950.
//
// A 1-D transform of length M along one axis of a strided array is done
// either in one pass (the whole sequence held in LDS) or by the four-step
// split M = L1 * L2 (two LDS passes with a twiddle between them).  In the
// four-step case the spectrum is left in "storage order": frequency
// k1 + L1 * k2 lives at position k1 * L2 + k2.  Every consumer of spectra in
// this library (the grid multiplier) is built by the same forward transform,
// so it is in the same order and the multiply is elementwise.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "common.h"

namespace sbd {

constexpr int kMaxStages = 16;

struct Radices {
  int n = 0;
  int r[kMaxStages];
};

// One LDS pass: FFTs of length L over a batch of sequences.
//   element e of sequence (inner b, outer o1, o2) is at
//   data + o2*sO2 + o1*sO1 + inner*1 + e*sE     with inner = ib*Bi + b.
// Zero padding on input: element is zero unless  e*lgE + o1*lgO + inner*lgI < n_in.
// Store only if the same logical index < n_out.
// Optional four-step twiddle W_M^(dir * e * q) with q = inner*twI + o1*twO, applied
// after the FFT (forward, tw_mode = 1) or before it (inverse, tw_mode = 2).
struct PassDesc {
  int L = 0;
  Radices rad;
  int64_t sE = 1, sO1 = 0, sO2 = 0;
  int Bi = 1;               // sequences per workgroup (a power of two)
  int lgBi = 0;             // log2(Bi), set by the launcher
  int64_t nInner = 1, nO1 = 1, nO2 = 1;
  int64_t lgE = 1, lgO = 0, lgI = 0;
  int64_t n_in = INT64_MAX, n_out = INT64_MAX;
  int tw_mode = 0;
  int64_t twI = 0, twO = 0, M = 1;
  int nthreads = 256;
  int ept = 8;
  size_t lds_bytes = 0;
  int xcd_remap = 0;          // 1: consecutive blocks of the inner dimension run on one XCD
};

// Plan for one axis of length M.
struct AxisPlan {
  int64_t M = 0;
  bool four_step = false;
  int L1 = 0, L2 = 0;        // four-step split (L1 * L2 = M); single pass: L1 = M
  Radices r1, r2, rs;
  void* twS = nullptr;       // two-level W_M table for the whole-column mode
  void* twSfull = nullptr;   // per-stage W tables of rs (read from global memory by the column pass)
  void* tw1 = nullptr;       // W_L1 table (T2)
  void* tw2 = nullptr;       // W_L2 table
  void* twM = nullptr;       // W_M table (four-step)
  bool is_double = false;
  int single_bi = 0;         // > 0: column transforms in one LDS pass holding single_bi columns
  int store_L1 = 0, store_L2 = 1;  // storage order of the spectrum: k1 * store_L2 + k2 holds k1 + store_L1 * k2
};

// Build radix decompositions and twiddle tables for an axis.  max_lds is the
// per-workgroup LDS budget in bytes, bi_rows the batch width used for strided
// passes (sequences per workgroup along the contiguous dimension).
int build_axis_plan(AxisPlan& ap, int64_t M, bool is_double, size_t max_lds, int bi_strided);
void free_axis_plan(AxisPlan& ap);

// True if n can be written with factors 2,3,5,7 only.
bool is_smooth(int64_t n);
int64_t next_smooth(int64_t n, int64_t multiple_of = 1);
int64_t best_fft_size(int64_t n, int64_t multiple_of = 1, bool is_double = false);

// Transform along the contiguous axis (rows) of a [nrows][pitch] complex array
// (batched over nbatch with stride sbatch).  dir = -1 forward, +1 inverse.
// n_in: input elements per row that may be non-zero (rest treated as zero);
// n_out: outputs stored per row (inverse only; forward stores all).
template <typename T>
int fft_rows(cplx<T>* data, int64_t nrows, int64_t pitch, int64_t nbatch, int64_t sbatch,
             const AxisPlan& ap, int dir, int64_t n_in, int64_t n_out, hipStream_t st);

// Transform along the strided axis (columns) of a [M][pitch] array, ncols columns.
// If mult != nullptr the last forward pass is fused with an elementwise
// multiply by mult (same storage layout as data; real if mult_complex == 0)
// and with the first inverse pass; the whole forward-multiply-inverse column
// sequence is then done and only rows < n_out are stored.
template <typename T>
int fft_cols(cplx<T>* data, int64_t ncols, int64_t pitch, int64_t nbatch, int64_t sbatch,
             const AxisPlan& ap, int dir, int64_t n_in, int64_t n_out,
             const void* mult, int mult_complex, int Bi, hipStream_t st);

// Real-data row transforms for the spread grid (Laplace kernel, real f).
// Forward: row y of the real grid F (assembled on load from the per-tile padded
// subgrids, overlaps summed) -> X[k], k = 0..M/2, through one complex FFT of
// length M/2 on z[j] = F[2j] + i F[2j+1].  Inverse: X[0..M/2] -> the first nx
// real values of the inverse DFT of length M (unnormalised), written as reals
// over the same row of `grid` (row pitch gpitch complex elements).
struct RealRowArgs {
  int64_t ny, nx, M;          // rows, valid real columns, real FFT length (even)
  int64_t gpitch;             // complex elements per grid row (>= M/2 + 1)
  int64_t nbatch, sbatch;     // right-hand sides, complex elements between grids
  // tile subgrid source (forward)
  const void* sub;            // [nbatch][ntiles][SG][SG] real T
  int T, SG, log2T;           // tile edge (a power of two), padded edge, log2(T)
  int64_t ntx, nty, ntiles;
  int pair = 0;               // compiled transforms: 1 = the spectra interleaved in row pairs
                              // (element (y, k) at ((y / 2) gpitch + k) 2 + y % 2), the inverse
                              // rows two per workgroup; the real output stays in natural rows
};
struct RealRowPlan {
  int64_t N = 0;              // M / 2
  Radices r;
  void* twN = nullptr;        // W_N table
  void* twM = nullptr;        // W_M^k, k = 0..N
  void* twS = nullptr;        // per-stage W tables of r
  bool is_double = false;
};
int build_real_row_plan(RealRowPlan& rp, int64_t M, bool is_double, size_t max_lds);
void free_real_row_plan(RealRowPlan& rp);
template <typename T>
int rows_r2c(cplx<T>* grid, const RealRowArgs& a, const RealRowPlan& rp, hipStream_t st);
template <typename T>
int rows_c2r(cplx<T>* grid, const RealRowArgs& a, const RealRowPlan& rp, hipStream_t st);

}  // namespace sbd
