// Device kernels of the SBD plan and apply (declarations of host launchers).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "common.h"

namespace sbd {

// Geometry and layout shared by plan and apply kernels.
struct Layout {
  int64_t n = 0;
  double x0 = 0, y0 = 0;      // tile-space origin (bounding-box minimum)
  double h = 0, inv_h = 0;    // x-grid spacing
  double inv_c = 0;           // inverse fine (near-field) cell size
  int T = 32;                 // tile edge (cells)
  int nsub = 1;               // fine cells per tile edge
  int64_t ntx = 0, nty = 0, ncx = 0, ncy = 0;
  int w = 7, PL = 4, SG = 40; // kernel width, pad, padded tile edge
  double beta = 0;
  int64_t nx = 0, ny = 0;     // spread grid (cells) = ntiles * T + 2 PL
  int64_t Mx = 0, My = 0;     // FFT sizes
  int64_t nkeys = 0;          // ntiles * nsub^2
};

// ---- plan kernels ----
int launch_bbox_partials(const double* pts, int64_t n, double* partials, int nblocks, hipStream_t st);
int launch_radius_partials(const double* pts, int64_t n, double cx, double cy, double* partials, int nblocks,
                           hipStream_t st);
int launch_keys(const double* pts, const Layout& L, int32_t* keys, int32_t* counts, int* bad, hipStream_t st);
int launch_scatter(const int32_t* keys, int64_t n, const int32_t* cell_start, int32_t* fill, int32_t* perm,
                   hipStream_t st);
int launch_sort_cells(const int32_t* cell_start, int64_t nkeys, int32_t* perm, hipStream_t st);
template <typename T>
int launch_gather_sorted(const double* pts, const int32_t* perm, const Layout& L, double2* xs,
                         typename cplx_of<T>::type* loc, int32_t* skeys, const int32_t* keys, hipStream_t st);
int launch_near_count(const double2* xt, const int32_t* tkeys, int64_t nt, const double2* xs,
                      const int32_t* cell_start, const Layout& L, double d2max, int self, int32_t* counts, int* dup,
                      hipStream_t st);
int launch_near_fill(const double2* xt, const int32_t* tkeys, int64_t nt, const double2* xs,
                     const int32_t* cell_start, const Layout& L, double d2max, int self, const int64_t* row_ptr,
                     int32_t* col, double* val, const double* chebA, const double* chebB, int deg, double U,
                     double self_re, int in_r, hipStream_t st);

// Frequency-side spreading of the concentric-circle nodes (plan-time Toeplitz symbol).
struct NodeSpreadArgs {
  const double* radius;        // per circle: |xi| (un-scaled, rad / length)
  const int64_t* M;            // per circle: nodes
  const double2* weight;       // per circle: complex weight per node (omega_hat)
  double h;                    // x-grid spacing
  const double* phihat_cheb;   // Chebyshev coefficients of phi_hat_1 on [0, tmax]
  int cheb_deg;
  double tmax;
  int64_t Kx, Ky;              // fine grid sizes
  int64_t sx, sy;              // output shift: fine mode g' holds H(g' + s) (weights times exp(i s . h xi))
  int wt;                      // psi width (cells)
  double beta_t;
  // storage order of the fine grid along each axis (four-step) : pos = (k % L1) * L2 + k / L1
  int64_t L1x, L2x, L1y, L2y;
  double2* grid;               // [Ky][Kx] complex128
};
// Spreading of the circle nodes onto the fine grid (type-1 NUFFT at plan time): one
// workgroup per kNodeTile x kNodeTile block of the fine grid gathers the nodes whose
// footprint reaches it (circles found by radius, nodes by angle), accumulates in LDS
// and writes its cells once (no global atomics, no clearing).  radius must be sorted
// ascending (with M and weight permuted alike).
constexpr int kNodeTile = 32;
int launch_node_gather(const NodeSpreadArgs& a, int ncirc, hipStream_t st);
// emb[Y][X] = H(|g_x|, |g_y|) for g = (X or X - Mx, Y or Y - My) inside |g_x| < nx, |g_y| < ny (H is
// even in each axis: every circle's node set is symmetric under xi_x -> -xi_x and xi_y -> -xi_y),
// read from fine mode (|g| - s) mod K and deconvolved by invpsi[| |g| - s |].
int launch_embed_symbol(const double2* fine, int64_t Kx, int64_t Ky, int64_t sx, int64_t sy, const double* invpsix,
                        const double* invpsiy, int64_t nx, int64_t ny, double2* emb, int64_t Mx, int64_t My,
                        hipStream_t st);
// Copy the FP64 symbol (in the storage order of an FP64 transform with splits
// (e1x, e2x), (e1y, e2y)) into the apply's storage order (splits (a1x, a2x), (a1y, a2y)),
// scaled, as real T (Laplace) or complex T (Helmholtz).
struct SymbolRemap {
  int64_t Mx, My;
  int64_t e1x, e2x, e1y, e2y;
  int64_t a1x, a2x, a1y, a2y;
};
template <typename T>
int launch_store_symbol(const double2* emb, const SymbolRemap& r, double scale, int complex_out, void* out,
                        hipStream_t st);

// Reorder a [My][Mx] complex array between natural frequency order and the
// four-step storage order (to_natural = 1: storage -> natural).
template <typename T>
int launch_reorder(const void* src, void* dst, int64_t Mx, int64_t My, int64_t L1x, int64_t L2x, int64_t L1y,
                   int64_t L2y, int to_natural, hipStream_t st);

// ---- plan: close-correction entries by the pair-difference NUFFT ----
// D_kl = G(y) - sum_nu omega_hat_nu exp(i y . xi_nu) at y = z_k - z_l on every stored pair
// (a type-3 NUFFT from the circle nodes xi to the pair differences y).  The nodes are
// spread with the ES kernel onto a G x G frequency grid of spacing h (cells j, centred
// index -G/2 <= j < G/2); at each y the grid's plane-wave sum is deconvolved by
// phi_hat(h y_x) phi_hat(h y_y).
struct PdArgs {
  const double* radius;        // per circle: |xi|
  const int64_t* node_start;   // [ncirc + 1]: first node of each circle
  const double2* weight;       // per circle: complex weight per node
  int ncirc;
  int64_t nnodes;
  int G;                       // frequency-grid edge, 8 <= G <= kPdMaxGrid, multiple of 8
  int J;                       // every non-zero cell has |j| <= J < G / 2
  double h;                    // frequency-grid spacing
  int w;                       // ES width (cells)
  double beta;
};
constexpr int kPdMaxGrid = 48;
// Number of per-wave partial grids launch_pd_spread writes for nnodes nodes.
int64_t pd_partials(int64_t nnodes);
// Spread every node onto partial grids [pd_partials][G][G] (row jy, column jx).
int launch_pd_spread(const PdArgs& a, double2* partials, hipStream_t st);
// Sum the partial grids in a fixed order into b [G][G].
int launch_pd_reduce(const double2* partials, int64_t nparts, int G, double2* b, hipStream_t st);
// Replace val[e] of every stored pair by the real part of G(y) - F(y), y = xt[row] - xs[col[e]]
// (F(0) alone on the diagonal of a single point set).  kind 0: G = -log|y| / (2 pi),
// kind 1: Re G = -Y0(k |y|) / 4.  phihat: Chebyshev coefficients of the ES transform on
// [0, tmax], tmax >= h |y_x|, h |y_y|.
int launch_pd_eval(const PdArgs& a, const double2* b, const double* phihat, int deg, double tmax, const double2* xt,
                   const double2* xs, const int64_t* row_ptr, const int32_t* col, int64_t nrows, int64_t nnz,
                   int self, int kind, double wavenumber, double* val, hipStream_t st);

// ---- apply kernels ----
// Interpolation work units: at most kUnitMaxPoints sorted points of one tile and
// about kUnitNnz close-correction entries (dense or long-row tiles are split).  A
// unit is processed in chunks of kUnitPoints points (512 points keep the
// workgroup's LDS near 16 KB, so eight workgroups fit on a CU).
constexpr int kUnitPoints = 512;
constexpr int kUnitMaxPoints = 2048;
constexpr int64_t kUnitNnz = 16384;
constexpr int kUnitMinPoints = 32;

struct ApplyArgs {
  const Layout* Ld;            // unused on device (host copy)
  int64_t n;
  int nrhs;
  int in_dtype;                // sbd_dtype of f and q
  int cplx_data;               // 1: complex f (complex grids), 0: real
  const void* f;
  void* q;
  const int32_t* perm;         // sources: sorted position -> input index
  const int32_t* tile_start;   // sources per tile
  int64_t nt;                  // number of targets (= n for a single point set)
  const int32_t* tperm;        // targets: sorted position -> output index
  const void* tloc;            // targets: tile-local offsets (cplx<T>)
  int self;                    // 1: targets are the sources (diagonal of D is the self term)
  const int32_t* unit_tile;    // interpolation work units: tile of unit u
  const int32_t* unit_start;   // [nunits + 1]: sorted-position range of unit u
  int64_t nunits;
  const void* loc;             // tile-local offsets (cplx<T> holding (ux, uy))
  int64_t ntiles;
  int T, w, PL, SG;
  double beta;
  int64_t ntx;
  void* sub;                   // per-tile padded subgrids
  void* fs;                    // sorted f copy
  void* grid;                  // complex FFT grid [My][Mx] per rhs
  int64_t Mx, My, nx, ny;
  const int64_t* row_ptr;
  const int32_t* col;
  const void* val;          // D values: double, or float when val_f32
  int val_f32;
  double self_im;
  int parts;
  int64_t nnz;
  int csr_group;               // lanes per CSR row (power of two, <= 64)
  int fs_inter;                // 1: the sorted f copy is laid out [n][nrhs] (else [nrhs][n])
  void* qnear;                 // non-null: D f of every right-hand side already summed per sorted
                               // target ([nrhs][nt] double or double2), added by the interpolation
  int real_grid;               // 1: the convolved grid is real T with row pitch 2 Mx
  int deterministic;           // 1: no float atomics (fixed-point FP64 spread, one-writer row sums)
  int sorted_io;               // 1: f read and q written in the plan's sorted order (no permutation)
};
template <typename T>
int launch_spread(const ApplyArgs& a, hipStream_t st);
template <typename T>
int launch_gather_grid(const ApplyArgs& a, hipStream_t st);
template <typename T>
int launch_interp_near(const ApplyArgs& a, hipStream_t st);
// Close correction of every right-hand side in one pass over D (nrhs > 1): one lane per
// (target, right-hand side); the lanes of a target read each entry once (one address) and
// the f values of all right-hand sides of its column as one contiguous run (fs_inter).
template <typename T>
int launch_near_multi(const ApplyArgs& a, hipStream_t st);
int launch_to_f32(const double* src, float* dst, int64_t n, hipStream_t st);

}  // namespace sbd
