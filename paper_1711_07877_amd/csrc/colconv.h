// Whole-column convolution pass with the transform length, radices and thread layout
// fixed at compile time (the hot pass of the far field: forward FFT along the
// zero-padded column, multiply by the grid symbol, inverse FFT, store the window).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "common.h"

namespace sbd {

namespace cc {
struct CcArgs {
  void* data;
  int64_t pitch;             // elements between rows
  int64_t ncols;
  int64_t sbatch;            // elements between right-hand sides
  int n_in, n_out;
  const void* tw;
  const void* sym;           // [Mx/2 + 1][L/2 + 1]
  int64_t mx;                // full row transform length (columns c > mx/2 read column mx - c)
  int ilv;                   // 1: row e at e * pitch; 2: rows interleaved in pairs, element (e, c)
                             //    at ((e / 2) * pitch + c) * 2 + e % 2
};
}  // namespace cc

struct ColConvPlan {
  int id = -1;               // compiled instance (-1: none for this length / precision)
  int64_t L = 0;             // column transform length
  void* tw = nullptr;        // device twiddle tables of the instance (forward and inverse stages)
  bool is_double = false;
  bool ch = false;           // complex symbol
};

// True if a compiled instance exists for length L in this precision and symbol type.
bool colconv_available(int64_t L, bool is_double, bool complex_symbol);
// Smallest compiled length >= n (0 if none).
int64_t colconv_size(int64_t n, bool is_double, bool complex_symbol);
// Builds the twiddle tables of the instance for L; returns 0, or -1 (no instance), -2 (memory).
int build_colconv_plan(ColConvPlan& cp, int64_t L, bool is_double, bool complex_symbol);
void free_colconv_plan(ColConvPlan& cp);

// For columns c < ncols of the [L][pitch] complex array data (one array per right-hand
// side, sbatch elements apart): rows e >= n_in are taken as zero, the column is
// transformed forward (exp(-2 pi i e k / L)), multiplied by the symbol, transformed back
// (unnormalised) and rows e < n_out are stored in place.  Requires n_in, n_out <= L / 2.
// sym: [Mx/2 + 1][L/2 + 1] real T (sym_complex = 0) or complex T; column c and frequency k
// read entry [min(c, Mx - c)][min(k, L - k)] (the symbol of a radial kernel on the symmetric
// grid window is even along both axes).  Mx is the full row transform length.
// ilv = 2: the rows are interleaved in pairs (element (e, c) at ((e / 2) * pitch + c) * 2 +
// e % 2), the layout of the paired real-row transforms; ilv = 1: natural rows.
template <typename T>
int colconv(cplx<T>* data, int64_t ncols, int64_t pitch, int64_t nbatch, int64_t sbatch, const ColConvPlan& cp,
            int64_t n_in, int64_t n_out, const void* sym, int sym_complex, int64_t Mx, int ilv, hipStream_t st);

// Plan time: the FP64 symbol emb ([My][Mx], each axis in the storage order of its transform,
// position of frequency k = (k % e1) * e2 + k / e1) to the column layout above, scaled, for
// the first ncols columns (frequencies kx) and rows ky <= My / 2.
template <typename T>
int store_symbol_cols(const double2* emb, int64_t Mx, int64_t My, int64_t ncols, int64_t e1x, int64_t e2x,
                      int64_t e1y, int64_t e2y, double scale, int complex_out, void* out, hipStream_t st);

}  // namespace sbd
