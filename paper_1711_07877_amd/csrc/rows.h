// Real-row transforms of the spread grid (Laplace, real f) with the row length, radices
// and thread layout fixed at compile time.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "common.h"
#include "fft.h"

namespace sbd {

namespace rr {
struct RowArgs {
  void* grid;                // complex rows, [nbatch][ny][gpitch]
  RealRowArgs a;
  const void* tw;            // stage twiddles: forward stages 1..3, inverse stages 1..3
  const void* twM;           // W_M^k, k = 0..N (M = 2 N)
};
}  // namespace rr

struct RowPlan {
  int id = -1;               // compiled instance (-1: none)
  int64_t N = 0;             // complex length (real length M = 2 N)
  void* tw = nullptr;
  void* twM = nullptr;
  bool is_double = false;
  bool pairs = false;        // instance with the two-rows-per-workgroup inverse (RealRowArgs::pair)
};

// Smallest compiled complex length >= n (0 if none).
int64_t rows_size(int64_t n, bool is_double);
// Builds the tables of the instance for N; 0, -1 (no instance), -2 (memory).
int build_row_plan(RowPlan& rp, int64_t N, bool is_double);
void free_row_plan(RowPlan& rp);

// Forward: row y of the real grid (assembled from the tile subgrids, overlaps summed)
// -> X[k], k = 0..N, of its real DFT of length M = 2 N, through one complex FFT of
// length N on z[j] = F[2j] + i F[2j+1].  Requires nx <= N (zero padding to M >= 2 nx).
template <typename T>
int rows_r2c_cc(cplx<T>* grid, const RealRowArgs& a, const RowPlan& rp, hipStream_t st);
// Inverse: X[0..N] -> the first nx real values of the unnormalised inverse real DFT of
// length M, written as reals over the same row.
template <typename T>
int rows_c2r_cc(cplx<T>* grid, const RealRowArgs& a, const RowPlan& rp, hipStream_t st);

}  // namespace sbd
