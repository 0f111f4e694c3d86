// Plan and apply kernels of the SBD matvec (gfx950).
#include <algorithm>
#include <cmath>
#include <cstdlib>

#include "devmath.h"
#include "kernels.h"

namespace sbd {

namespace {

constexpr int kBlock = 256;

// ---------------------------------------------------------------- plan: geometry
__global__ void k_bbox(const double* __restrict__ pts, int64_t n, double* partials) {
  __shared__ double s[4][kBlock];
  double mnx = INFINITY, mny = INFINITY, mxx = -INFINITY, mxy = -INFINITY;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    double x = pts[2 * i], y = pts[2 * i + 1];
    mnx = fmin(mnx, x); mny = fmin(mny, y); mxx = fmax(mxx, x); mxy = fmax(mxy, y);
  }
  s[0][threadIdx.x] = mnx; s[1][threadIdx.x] = mny; s[2][threadIdx.x] = mxx; s[3][threadIdx.x] = mxy;
  __syncthreads();
  for (int st = blockDim.x / 2; st > 0; st >>= 1) {
    if (threadIdx.x < st) {
      s[0][threadIdx.x] = fmin(s[0][threadIdx.x], s[0][threadIdx.x + st]);
      s[1][threadIdx.x] = fmin(s[1][threadIdx.x], s[1][threadIdx.x + st]);
      s[2][threadIdx.x] = fmax(s[2][threadIdx.x], s[2][threadIdx.x + st]);
      s[3][threadIdx.x] = fmax(s[3][threadIdx.x], s[3][threadIdx.x + st]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int k = 0; k < 4; ++k) partials[4 * blockIdx.x + k] = s[k][0];
}

__global__ void k_radius(const double* __restrict__ pts, int64_t n, double cx, double cy, double* partials) {
  __shared__ double s[kBlock];
  double m = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    double dx = pts[2 * i] - cx, dy = pts[2 * i + 1] - cy;
    m = fmax(m, dx * dx + dy * dy);
  }
  s[threadIdx.x] = m;
  __syncthreads();
  for (int st = blockDim.x / 2; st > 0; st >>= 1) {
    if (threadIdx.x < st) s[threadIdx.x] = fmax(s[threadIdx.x], s[threadIdx.x + st]);
    __syncthreads();
  }
  if (threadIdx.x == 0) partials[blockIdx.x] = s[0];
}

// ---------------------------------------------------------------- plan: binning
struct KeyArgs {
  double x0, y0, inv_c;
  int64_t ncx, ncy, ntx;
  int nsub;
};

__global__ void k_keys(const double* __restrict__ pts, int64_t n, KeyArgs a, int32_t* keys, int32_t* counts, int* bad) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  double x = pts[2 * i], y = pts[2 * i + 1];
  if (!(x == x) || !(y == y) || isinf(x) || isinf(y)) {
    atomicOr(bad, 1);
    keys[i] = 0;
    atomicAdd(&counts[0], 1);
    return;
  }
  double fxd = floor(__dmul_rn(__dsub_rn(x, a.x0), a.inv_c));
  double fyd = floor(__dmul_rn(__dsub_rn(y, a.y0), a.inv_c));
  fxd = fxd < 0.0 ? 0.0 : (fxd > (double)(a.ncx - 1) ? (double)(a.ncx - 1) : fxd);
  fyd = fyd < 0.0 ? 0.0 : (fyd > (double)(a.ncy - 1) ? (double)(a.ncy - 1) : fyd);
  int64_t fx = (int64_t)fxd, fy = (int64_t)fyd;
  int64_t tile = (fy / a.nsub) * a.ntx + (fx / a.nsub);
  int64_t key = tile * a.nsub * a.nsub + (fy % a.nsub) * a.nsub + (fx % a.nsub);
  keys[i] = (int32_t)key;
  atomicAdd(&counts[key], 1);
}

__global__ void k_scatter(const int32_t* __restrict__ keys, int64_t n, const int32_t* __restrict__ cell_start,
                          int32_t* fill, int32_t* perm) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  int32_t k = keys[i];
  int32_t pos = cell_start[k] + atomicAdd(&fill[k], 1);
  perm[pos] = (int32_t)i;
}

__device__ void sift_down(int32_t* a, int64_t root, int64_t end) {
  while (2 * root + 1 < end) {
    int64_t c = 2 * root + 1;
    if (c + 1 < end && a[c] < a[c + 1]) ++c;
    if (a[root] < a[c]) {
      int32_t t = a[root]; a[root] = a[c]; a[c] = t;
      root = c;
    } else {
      return;
    }
  }
}

// Order each cell's points by input index: the scatter above is a counting sort by
// key whose order inside a key depends on atomics; sorting inside the cell makes
// the whole permutation the stable sort by key.
__global__ void k_sort_cells(const int32_t* __restrict__ cell_start, int64_t nkeys, int32_t* perm) {
  int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (c >= nkeys) return;
  int64_t s = cell_start[c], e = cell_start[c + 1];
  int64_t m = e - s;
  if (m < 2) return;
  int32_t* a = perm + s;
  if (m <= 48) {
    for (int64_t i = 1; i < m; ++i) {
      int32_t v = a[i];
      int64_t j = i - 1;
      while (j >= 0 && a[j] > v) { a[j + 1] = a[j]; --j; }
      a[j + 1] = v;
    }
    return;
  }
  for (int64_t r = m / 2 - 1; r >= 0; --r) sift_down(a, r, m);
  for (int64_t end = m - 1; end > 0; --end) {
    int32_t t = a[0]; a[0] = a[end]; a[end] = t;
    sift_down(a, 0, end);
  }
}

struct GatherArgs {
  double x0, y0, inv_h;
  int T, nsub;
  int64_t ntx;
};

template <typename T>
__global__ void k_gather_sorted(const double* __restrict__ pts, const int32_t* __restrict__ perm, int64_t n,
                                GatherArgs a, double2* xs, cplx<T>* loc, int32_t* skeys,
                                const int32_t* __restrict__ keys) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  int32_t o = perm[i];
  double x = pts[2 * o], y = pts[2 * o + 1];
  int32_t key = keys[o];
  skeys[i] = key;
  xs[i] = make_double2(x, y);
  int64_t tile = key / (a.nsub * a.nsub);
  int64_t tx = tile % a.ntx, ty = tile / a.ntx;
  double ux = (x - a.x0) * a.inv_h - (double)(tx * a.T);
  double uy = (y - a.y0) * a.inv_h - (double)(ty * a.T);
  const double top = (double)a.T * (1.0 - (sizeof(T) == 4 ? 6.0e-8 : 2.3e-16));
  ux = ux < 0.0 ? 0.0 : (ux > top ? top : ux);
  uy = uy < 0.0 ? 0.0 : (uy > top ? top : uy);
  T fx = (T)ux, fy = (T)uy;
  if (fx >= (T)a.T) fx = (T)top;
  if (fy >= (T)a.T) fy = (T)top;
  loc[i] = mk<T>(fx, fy);
}

// ---------------------------------------------------------------- plan: near field
struct NearArgs {
  int64_t n;
  int nsub;
  int64_t ntx, ncx, ncy;
  double d2max;
};

__device__ __forceinline__ int neighbour_keys(int32_t key, const NearArgs& a, int32_t* nk) {
  int64_t ns2 = (int64_t)a.nsub * a.nsub;
  int64_t t = key / ns2, sub = key % ns2;
  int64_t fx = (t % a.ntx) * a.nsub + sub % a.nsub;
  int64_t fy = (t / a.ntx) * a.nsub + sub / a.nsub;
  int cnt = 0;
  for (int dy = -1; dy <= 1; ++dy) {
    int64_t gy = fy + dy;
    if (gy < 0 || gy >= a.ncy) continue;
    for (int dx = -1; dx <= 1; ++dx) {
      int64_t gx = fx + dx;
      if (gx < 0 || gx >= a.ncx) continue;
      int64_t tt = (gy / a.nsub) * a.ntx + gx / a.nsub;
      nk[cnt++] = (int32_t)(tt * ns2 + (gy % a.nsub) * a.nsub + gx % a.nsub);
    }
  }
  for (int i = 1; i < cnt; ++i) {  // ascending keys = ascending sorted positions
    int32_t v = nk[i];
    int j = i - 1;
    while (j >= 0 && nk[j] > v) { nk[j + 1] = nk[j]; --j; }
    nk[j + 1] = v;
  }
  return cnt;
}

struct FillArgs {
  const double* chebA;
  const double* chebB;
  int deg;
  double U;
  double self_re;
  int in_r;          // tables in r = sqrt(u) on [0, sqrt(U)] instead of u on [0, U]
};

// Pairs (target i, source j) with d2 <= delta_min^2: xt/tkeys are the sorted targets,
// xs/cell_start the sorted sources (the same arrays for a single point set, where
// self = 1 marks i == j as the diagonal; otherwise any d2 == 0 is a coincidence).
//
// 16 consecutive lanes share one row and walk its candidate sources 16 at a
// time (curves put hundreds of candidates in the 3 x 3 cells of a point); the lanes'
// matches are ranked with the group's ballot bits, so the row keeps ascending columns
// and every group writes its entries as consecutive runs.
constexpr int kNearGroup = 16;

__device__ __forceinline__ uint32_t group_bits(bool pred) {
  const uint64_t b = __ballot(pred);
  const int base = (threadIdx.x & 63) & ~(kNearGroup - 1);
  return (uint32_t)((b >> base) & ((1ull << kNearGroup) - 1));
}

__global__ void __launch_bounds__(256) k_near_count_g(const double2* __restrict__ xt, const int32_t* __restrict__ tkeys,
                                                       const double2* __restrict__ xs,
                                                       const int32_t* __restrict__ cell_start, NearArgs a, int self,
                                                       int32_t* counts, int* dup) {
  const int64_t i = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / kNearGroup;
  const int g = threadIdx.x & (kNearGroup - 1);
  const bool live = i < a.n;  // whole groups are live or not: blockDim is a multiple of the group
  double2 p = make_double2(0.0, 0.0);
  int32_t nk[9];
  int cnt = 0;
  if (live) {
    p = xt[i];
    cnt = neighbour_keys(tkeys[i], a, nk);
  }
  int32_t c = 0;
  for (int k = 0; k < cnt; ++k) {
    const int32_t s = cell_start[nk[k]], e = cell_start[nk[k] + 1];
    for (int32_t j0 = s; j0 < e; j0 += kNearGroup) {
      const int32_t j = j0 + g;
      bool hit = false;
      if (j < e) {
        const double2 q = xs[j];
        const double d2 = d2_exact(p.x, p.y, q.x, q.y);
        hit = d2 <= a.d2max;
        if (hit && d2 == 0.0 && (!self || j != i)) atomicOr(dup, 1);
      }
      c += __popc(group_bits(hit));
    }
  }
  if (live && g == 0) counts[i] = c;
}

__global__ void __launch_bounds__(256) k_near_fill_g(const double2* __restrict__ xt, const int32_t* __restrict__ tkeys,
                                                      const double2* __restrict__ xs,
                                                      const int32_t* __restrict__ cell_start, NearArgs a, int self,
                                                      const int64_t* __restrict__ row_ptr, int32_t* col, double* val,
                                                      FillArgs fa) {
  const int64_t i = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / kNearGroup;
  const int g = threadIdx.x & (kNearGroup - 1);
  const bool live = i < a.n;
  double2 p = make_double2(0.0, 0.0);
  int32_t nk[9];
  int cnt = 0;
  int64_t o = 0;
  if (live) {
    p = xt[i];
    cnt = neighbour_keys(tkeys[i], a, nk);
    o = row_ptr[i];
  }
  const uint32_t below = (1u << g) - 1u;
  for (int k = 0; k < cnt; ++k) {
    const int32_t s = cell_start[nk[k]], e = cell_start[nk[k] + 1];
    for (int32_t j0 = s; j0 < e; j0 += kNearGroup) {
      const int32_t j = j0 + g;
      bool hit = false;
      double d2 = 0.0;
      if (j < e) {
        const double2 q = xs[j];
        d2 = d2_exact(p.x, p.y, q.x, q.y);
        hit = d2 <= a.d2max;
      }
      const uint32_t bits = group_bits(hit);
      if (hit) {
        const int64_t at = o + __popc(bits & below);
        col[at] = j;
        double v;
        if (self && j == i) {
          v = fa.self_re;
        } else {
          const double t = fa.in_r ? 2.0 * sqrt(d2 / fa.U) - 1.0 : 2.0 * d2 / fa.U - 1.0;
          v = cheb_eval(fa.chebA, fa.deg, t) * log(d2) + cheb_eval(fa.chebB, fa.deg, t);
        }
        val[at] = v;
      }
      o += __popc(bits);
    }
  }
}

// ---------------------------------------------------------------- plan: Toeplitz symbol
constexpr int kGatherCircles = 1024;  // circles handled per batch in one tile

__device__ __forceinline__ double wrap_pi(double a) {
  const double tp = 6.283185307179586476925;
  while (a > 3.141592653589793238463) a -= tp;
  while (a <= -3.141592653589793238463) a += tp;
  return a;
}

__global__ void __launch_bounds__(256) k_node_gather(NodeSpreadArgs a, int ncirc) {
  __shared__ double2 acc[kNodeTile * kNodeTile];
  __shared__ int cpid[kGatherCircles];
  __shared__ int64_t cm0[kGatherCircles];
  __shared__ int cstart[kGatherCircles + 1];
  const int64_t i0 = (int64_t)blockIdx.x * kNodeTile - a.Kx / 2;  // centred cell indices
  const int64_t j0 = (int64_t)blockIdx.y * kNodeTile - a.Ky / 2;
  for (int c = threadIdx.x; c < kNodeTile * kNodeTile; c += blockDim.x) acc[c] = make_double2(0.0, 0.0);
  // nodes reaching the tile: node coordinate v (cells) in (i0 - wt/2, i0 + TB - 1 + wt/2]
  const double hw = 0.5 * a.wt;
  const double ex0 = (double)i0 - hw, ex1 = (double)(i0 + kNodeTile - 1) + hw;
  const double ey0 = (double)j0 - hw, ey1 = (double)(j0 + kNodeTile - 1) + hw;
  const double inv2pi = 0.15915494309189533577;
  const double sx = 1.0 / (a.h * inv2pi * (double)a.Kx), sy = 1.0 / (a.h * inv2pi * (double)a.Ky);
  const double bx0 = ex0 * sx, bx1 = ex1 * sx, by0 = ey0 * sy, by1 = ey1 * sy;  // physical box
  const double dx = bx0 > 0 ? bx0 : (bx1 < 0 ? -bx1 : 0.0);
  const double dy = by0 > 0 ? by0 : (by1 < 0 ? -by1 : 0.0);
  const double rmin = sqrt(dx * dx + dy * dy);
  const double mx = fmax(fabs(bx0), fabs(bx1)), my = fmax(fabs(by0), fabs(by1));
  const double rmax = sqrt(mx * mx + my * my);
  const bool full = (bx0 <= 0 && bx1 >= 0 && by0 <= 0 && by1 >= 0);
  double tlo = 0, thi = 0;
  if (!full) {
    const double tc = atan2(0.5 * (by0 + by1), 0.5 * (bx0 + bx1));
    double dmin = 0, dmax = 0;
    const double cx[4] = {bx0, bx1, bx0, bx1}, cy[4] = {by0, by0, by1, by1};
    for (int q = 0; q < 4; ++q) {
      double d = wrap_pi(atan2(cy[q], cx[q]) - tc);
      dmin = q ? fmin(dmin, d) : d;
      dmax = q ? fmax(dmax, d) : d;
    }
    tlo = tc + dmin;
    thi = tc + dmax;
  }
  // circles with rmin <= radius <= rmax (radius sorted ascending)
  int lo = 0, hi = ncirc;
  while (lo < hi) { int mid = (lo + hi) >> 1; if (a.radius[mid] < rmin * (1 - 1e-12)) lo = mid + 1; else hi = mid; }
  const int pa = lo;
  lo = pa; hi = ncirc;
  while (lo < hi) { int mid = (lo + hi) >> 1; if (a.radius[mid] <= rmax * (1 + 1e-12)) lo = mid + 1; else hi = mid; }
  const int pb = lo;
  const double tw = 2.0 / a.wt;
  const double h2 = a.h * a.h;
  for (int cb = pa; cb < pb; cb += kGatherCircles) {
    const int nc = min(kGatherCircles, pb - cb);
    __syncthreads();
    for (int c = threadIdx.x; c < nc; c += blockDim.x) {
      const int p = cb + c;
      const int64_t Mp = a.M[p];
      int64_t m0 = 0, cnt = Mp;
      if (!full) {
        const double f = (double)Mp * inv2pi;
        int64_t mlo = (int64_t)floor(tlo * f) - 1, mhi = (int64_t)ceil(thi * f) + 1;
        if (mhi - mlo + 1 < Mp) { m0 = mlo; cnt = mhi - mlo + 1; }
      }
      cpid[c] = p;
      cm0[c] = m0;
      cstart[c + 1] = (int)cnt;
    }
    __syncthreads();
    if (threadIdx.x == 0) {  // exclusive prefix over at most kGatherCircles counts
      cstart[0] = 0;
      for (int c = 0; c < nc; ++c) cstart[c + 1] += cstart[c];
    }
    __syncthreads();
    const int total = cstart[nc];
    for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
      int l = 0, r = nc;  // circle c with cstart[c] <= idx < cstart[c + 1]
      while (r - l > 1) { int mid = (l + r) >> 1; if (cstart[mid] <= idx) l = mid; else r = mid; }
      const int p = cpid[l];
      const int64_t Mp = a.M[p];
      int64_t m = cm0[l] + (idx - cstart[l]);
      m %= Mp;
      if (m < 0) m += Mp;
      const double R = a.radius[p];
      double sn, cs;
      sincospi(2.0 * (double)m / (double)Mp, &sn, &cs);
      const double xi_x = R * cs, xi_y = R * sn;
      const double vx = a.h * xi_x * inv2pi * (double)a.Kx;
      const double vy = a.h * xi_y * inv2pi * (double)a.Ky;
      const int64_t ix0 = (int64_t)floor(vx - hw) + 1, iy0 = (int64_t)floor(vy - hw) + 1;
      const int64_t ka = max(ix0, i0), kb = min(ix0 + a.wt, i0 + kNodeTile);
      const int64_t la = max(iy0, j0), lb = min(iy0 + a.wt, j0 + kNodeTile);
      if (ka >= kb || la >= lb) continue;
      const double tx = 2.0 * fabs(xi_x) / a.tmax - 1.0;
      const double ty = 2.0 * fabs(xi_y) / a.tmax - 1.0;
      const double phx = cheb_eval(a.phihat_cheb, a.cheb_deg, tx);
      const double phy = cheb_eval(a.phihat_cheb, a.cheb_deg, ty);
      const double sc = h2 * h2 / ((phx * phy) * (phx * phy));
      const double2 wgt = a.weight[p];
      // shift of the output window: weight times exp(i h (sx xi_x + sy xi_y))
      double ss, sc2;
      sincos(a.h * ((double)a.sx * xi_x + (double)a.sy * xi_y), &ss, &sc2);
      const double cr = (wgt.x * sc2 - wgt.y * ss) * sc, ci = (wgt.x * ss + wgt.y * sc2) * sc;
      double px[16];
      const int nxk = (int)(kb - ka);
      for (int k = 0; k < nxk; ++k) px[k] = es_kernel<double>((double)(ka + k) - vx, tw, a.beta_t);
      for (int64_t iy = la; iy < lb; ++iy) {
        const double py = es_kernel<double>((double)iy - vy, tw, a.beta_t);
        double* rowp = reinterpret_cast<double*>(acc + (iy - j0) * kNodeTile) + 2 * (ka - i0);
        for (int k = 0; k < nxk; ++k) {
          const double w = px[k] * py;
          atomicAdd(rowp + 2 * k, cr * w);
          atomicAdd(rowp + 2 * k + 1, ci * w);
        }
      }
    }
  }
  __syncthreads();
  for (int c = threadIdx.x; c < kNodeTile * kNodeTile; c += blockDim.x) {
    const int64_t i = i0 + (c % kNodeTile), j = j0 + (c / kNodeTile);
    if (i >= a.Kx - a.Kx / 2 || j >= a.Ky - a.Ky / 2) continue;  // beyond the last centred index
    const int64_t kx = i < 0 ? i + a.Kx : i, ky = j < 0 ? j + a.Ky : j;
    const int64_t px = (kx % a.L1x) * a.L2x + kx / a.L1x;
    const int64_t py = (ky % a.L1y) * a.L2y + ky / a.L1y;
    a.grid[py * a.Kx + px] = acc[c];
  }
}



__global__ void k_embed(const double2* __restrict__ fine, int64_t Kx, int64_t Ky, int64_t sx, int64_t sy,
                        const double* __restrict__ ipx, const double* __restrict__ ipy, int64_t nx, int64_t ny,
                        double2* emb, int64_t Mx, int64_t My) {
  int64_t X = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  int64_t Y = blockIdx.y;
  if (X >= Mx || Y >= My) return;
  int64_t gx = X < nx ? X : (X > Mx - nx ? Mx - X : INT64_MIN);  // |g_x|
  int64_t gy = Y < ny ? Y : (Y > My - ny ? My - Y : INT64_MIN);
  double2 v = make_double2(0.0, 0.0);
  if (gx != INT64_MIN && gy != INT64_MIN) {
    const int64_t mx = gx - sx, my = gy - sy;  // fine modes
    const int64_t kx = ((mx % Kx) + Kx) % Kx, ky = ((my % Ky) + Ky) % Ky;
    double2 f = fine[ky * Kx + kx];
    double s = ipx[mx < 0 ? -mx : mx] * ipy[my < 0 ? -my : my];
    v = make_double2(f.x * s, f.y * s);
  }
  emb[Y * Mx + X] = v;
}

__device__ __forceinline__ int64_t pos_to_freq(int64_t pos, int64_t L1, int64_t L2) {
  // storage position k1 * L2 + k2 holds frequency k1 + L1 * k2
  return pos / L2 + L1 * (pos % L2);
}
__device__ __forceinline__ int64_t freq_to_pos(int64_t k, int64_t L1, int64_t L2) {
  return (k % L1) * L2 + k / L1;
}

template <typename T>
__global__ void k_store_symbol(const double2* __restrict__ emb, SymbolRemap r, double scale, int complex_out, void* out) {
  int64_t X = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  int64_t Y = blockIdx.y;
  if (X >= r.Mx) return;
  int64_t kx = pos_to_freq(X, r.a1x, r.a2x), ky = pos_to_freq(Y, r.a1y, r.a2y);
  int64_t src = freq_to_pos(ky, r.e1y, r.e2y) * r.Mx + freq_to_pos(kx, r.e1x, r.e2x);
  double2 v = emb[src];
  int64_t i = Y * r.Mx + X;
  if (complex_out) reinterpret_cast<cplx<T>*>(out)[i] = mk<T>((T)(v.x * scale), (T)(v.y * scale));
  else reinterpret_cast<T*>(out)[i] = (T)(v.x * scale);
}

template <typename T>
__global__ void k_reorder(const cplx<T>* __restrict__ src, cplx<T>* dst, int64_t Mx, int64_t My, int64_t L1x,
                          int64_t L2x, int64_t L1y, int64_t L2y, int to_natural) {
  int64_t X = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  int64_t Y = blockIdx.y;
  if (X >= Mx) return;
  int64_t px = freq_to_pos(X, L1x, L2x), py = freq_to_pos(Y, L1y, L2y);
  if (to_natural) dst[Y * Mx + X] = src[py * Mx + px];
  else dst[py * Mx + px] = src[Y * Mx + X];
}

// ---------------------------------------------------------------- apply
__device__ __forceinline__ void load_f(const void* f, int dtype, int64_t idx, double& re, double& im) {
  switch (dtype) {
    case 0: re = reinterpret_cast<const double*>(f)[idx]; im = 0.0; break;
    case 1: re = reinterpret_cast<const float*>(f)[idx]; im = 0.0; break;
    case 2: { double2 v = reinterpret_cast<const double2*>(f)[idx]; re = v.x; im = v.y; } break;
    default: { float2 v = reinterpret_cast<const float2*>(f)[idx]; re = v.x; im = v.y; } break;
  }
}

__device__ __forceinline__ void store_q(void* q, int dtype, int64_t idx, double re, double im) {
  switch (dtype) {
    case 0: reinterpret_cast<double*>(q)[idx] = re; break;
    case 1: reinterpret_cast<float*>(q)[idx] = (float)re; break;
    case 2: reinterpret_cast<double2*>(q)[idx] = make_double2(re, im); break;
    default: reinterpret_cast<float2*>(q)[idx] = make_float2((float)re, (float)im); break;
  }
}

// position of sorted point i, right-hand side r, in the sorted f copy
__device__ __forceinline__ int64_t fs_idx(const ApplyArgs& a, int r, int64_t i) {
  return a.fs_inter ? i * a.nrhs + r : (int64_t)r * a.n + i;
}

// Spread (z, f) of one tile into its padded (T + 2 PL)^2 subgrid in LDS with the
// exponential-of-semicircle kernel, then store the subgrid (no cross-tile atomics;
// overlapping halos are summed when the FFT grid is assembled).
//
// FP64 plans: the LDS accumulators are FP64 (on gfx950 ds_add_f64 sustains about 7
// lane-updates per clock per CU while ds_add_f32 sustains about 0.3).  Points are sorted by
// fine cell, so neighbouring sorted points have nearly identical footprints; to keep
// one instruction's addresses apart the 64 lanes of a wave take points spread over
// the tile's sorted list (a 64 x R transpose of the processing order) and each lane
// walks the rows of its footprint starting at a lane-dependent row.
template <typename T, bool CPLX>
__global__ void __launch_bounds__(256) k_spread(ApplyArgs a) {
  extern __shared__ unsigned char smem_raw[];
  double* sre = reinterpret_cast<double*>(smem_raw);
  double* sim = sre + a.SG * a.SG;
  const int64_t t = blockIdx.x;
  const int r = blockIdx.y;
  const int SG2 = a.SG * a.SG;
  for (int k = threadIdx.x; k < SG2; k += blockDim.x) {
    sre[k] = 0.0;
    if (CPLX) sim[k] = 0.0;
  }
  __syncthreads();
  const int32_t s = a.tile_start[t], e = a.tile_start[t + 1];
  const int cnt = e - s;
  const int R = (cnt + 63) / 64;
  const cplx<T>* loc = reinterpret_cast<const cplx<T>*>(a.loc);
  const T two_over_w = T(2) / T(a.w);
  const T beta = (T)a.beta;
  const T halfw = T(0.5) * T(a.w);
  const int lane = threadIdx.x & 63;
  for (int kk = threadIdx.x; kk < 64 * R; kk += blockDim.x) {
    const int p = (kk & 63) * R + (kk >> 6);
    if (p >= cnt) continue;
    const int32_t i = s + p;
    double fr, fi;
    load_f(a.f, a.in_dtype, (int64_t)r * a.n + (a.sorted_io ? i : a.perm[i]), fr, fi);
    T vr = (T)fr, vi = (T)fi;
    if (CPLX) reinterpret_cast<cplx<T>*>(a.fs)[fs_idx(a, r, i)] = mk<T>(vr, vi);
    else reinterpret_cast<T*>(a.fs)[fs_idx(a, r, i)] = vr;
    cplx<T> u = loc[i];
    int jx0 = (int)floor(u.x - halfw) + 1;
    int jy0 = (int)floor(u.y - halfw) + 1;
    T wx[16];
    for (int k = 0; k < a.w; ++k) wx[k] = es_kernel<T>(T(jx0 + k) - u.x, two_over_w, beta);
    int b = lane % a.w;
    for (int jb = 0; jb < a.w; ++jb) {
      T wyb = es_kernel<T>(T(jy0 + b) - u.y, two_over_w, beta);
      int rowoff = (jy0 + b + a.PL) * a.SG + jx0 + a.PL;
      T vyr = vr * wyb;
      T vyi = vi * wyb;
      for (int k = 0; k < a.w; ++k) {
        atomicAdd(&sre[rowoff + k], (double)(vyr * wx[k]));
        if (CPLX) atomicAdd(&sim[rowoff + k], (double)(vyi * wx[k]));
      }
      b = (b + 1 == a.w) ? 0 : b + 1;
    }
  }
  __syncthreads();
  T* out = reinterpret_cast<T*>(a.sub) + ((int64_t)r * a.ntiles + t) * (int64_t)SG2 * (CPLX ? 2 : 1);
  for (int k = threadIdx.x; k < SG2; k += blockDim.x) {
    if (CPLX) {
      out[2 * k] = (T)sre[k];
      out[2 * k + 1] = (T)sim[k];
    } else {
      out[k] = (T)sre[k];
    }
  }
}

// FP32 plans: the tile accumulates in 32-bit fixed point with ds_add_u32 (about 13
// lane-updates per clock per CU, against about 7 for ds_add_f64).  A first pass over
// the tile's points forms S = sum |f| per component; every contribution is
// f phi(x) phi(y) with |phi| <= 1, so any cell sum is bounded by S and the scale
// 2^29 / S keeps every accumulator, rounding included, inside int32.  The absolute
// resolution S / 2^29 is about 1e-6 of a typical cell value, and integer sums do not
// depend on the order of the atomic updates, so the grid is reproducible.
// One point's W x W footprint into the fixed-point tile (rows taken from a
// lane-dependent start so that one instruction's lanes hit different rows).
template <typename T, bool CPLX, int W>
__device__ __forceinline__ void spread_point_fixed(int* ire, int* iim, int SG, int PL, cplx<T> u, float vr, float vi,
                                                   T two_over_w, T beta, int lane) {
  const T halfw = T(0.5) * T(W);
  const int jx0 = (int)floor(u.x - halfw) + 1;
  const int jy0 = (int)floor(u.y - halfw) + 1;
  float wx[W];
#pragma unroll
  for (int k = 0; k < W; ++k) wx[k] = (float)es_kernel<T>(T(jx0 + k) - u.x, two_over_w, beta);
  int b = lane % W;
  for (int jb = 0; jb < W; ++jb) {
    const float wyb = (float)es_kernel<T>(T(jy0 + b) - u.y, two_over_w, beta);
    const int rowoff = (jy0 + b + PL) * SG + jx0 + PL;
    const float vyr = vr * wyb;
    const float vyi = vi * wyb;
#pragma unroll
    for (int k = 0; k < W; ++k) {
      atomicAdd(&ire[rowoff + k], __float2int_rn(vyr * wx[k]));
      if (CPLX) atomicAdd(&iim[rowoff + k], __float2int_rn(vyi * wx[k]));
    }
    b = (b + 1 == W) ? 0 : b + 1;
  }
}

template <typename T, bool CPLX>
__global__ void __launch_bounds__(256) k_spread_fixed(ApplyArgs a) {
  extern __shared__ unsigned char smem_raw[];
  int* ire = reinterpret_cast<int*>(smem_raw);
  int* iim = ire + a.SG * a.SG;
  __shared__ float red[2][256 / 64];
  const int64_t t = blockIdx.x;
  const int r = blockIdx.y;
  const int SG2 = a.SG * a.SG;
  for (int k = threadIdx.x; k < SG2; k += blockDim.x) {
    ire[k] = 0;
    if (CPLX) iim[k] = 0;
  }
  const int32_t s = a.tile_start[t], e = a.tile_start[t + 1];
  const int cnt = e - s;
  const int R = (cnt + 63) / 64;
  // pass 1: gather f into sorted order (kept for the close correction) and sum |f|;
  // each thread visits the same points as in pass 2, so pass 2 reads back its own stores
  float sr = 0.f, si = 0.f;
  for (int kk = threadIdx.x; kk < 64 * R; kk += blockDim.x) {
    const int p = (kk & 63) * R + (kk >> 6);
    if (p >= cnt) continue;
    const int32_t i = s + p;
    double fr, fi;
    load_f(a.f, a.in_dtype, (int64_t)r * a.n + (a.sorted_io ? i : a.perm[i]), fr, fi);
    T vr = (T)fr, vi = (T)fi;
    if (CPLX) reinterpret_cast<cplx<T>*>(a.fs)[fs_idx(a, r, i)] = mk<T>(vr, vi);
    else reinterpret_cast<T*>(a.fs)[fs_idx(a, r, i)] = vr;
    sr += fabsf((float)vr);
    si += fabsf((float)vi);
  }
  for (int off = 32; off > 0; off >>= 1) {
    sr += __shfl_down(sr, off, 64);
    si += __shfl_down(si, off, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    red[0][threadIdx.x >> 6] = sr;
    red[1][threadIdx.x >> 6] = si;
  }
  __syncthreads();
  float tr = 0.f, ti = 0.f;
  for (int k = 0; k < (int)(blockDim.x >> 6); ++k) {
    tr += red[0][k];
    ti += red[1][k];
  }
  T* out = reinterpret_cast<T*>(a.sub) + ((int64_t)r * a.ntiles + t) * (int64_t)SG2 * (CPLX ? 2 : 1);
  if (!(tr <= 3.0e38f) || !(ti <= 3.0e38f)) {
    // a non-finite f (or a sum beyond the FP32 range): no fixed-point scale exists, and a
    // floating-point spread would carry NaN/inf into the grid, so the tile is written as NaN
    // (the far field then makes every q NaN).  tr, ti are the same in every thread.
    const T nanv = __builtin_nan("");
    for (int k = threadIdx.x; k < SG2 * (CPLX ? 2 : 1); k += blockDim.x) out[k] = nanv;
    return;
  }
  // 1.01 covers the rounding of the float sums above
  const float scr = tr > 0.f ? 536870912.0f / (1.01f * tr) : 1.0f;
  const float sci = ti > 0.f ? 536870912.0f / (1.01f * ti) : 1.0f;
  const cplx<T>* loc = reinterpret_cast<const cplx<T>*>(a.loc);
  const T two_over_w = T(2) / T(a.w);
  const T beta = (T)a.beta;
  const T halfw = T(0.5) * T(a.w);
  const int lane = threadIdx.x & 63;
  for (int kk = threadIdx.x; kk < 64 * R; kk += blockDim.x) {
    const int p = (kk & 63) * R + (kk >> 6);
    if (p >= cnt) continue;
    const int32_t i = s + p;
    float vr, vi = 0.f;
    if (CPLX) {
      cplx<T> fv = reinterpret_cast<const cplx<T>*>(a.fs)[fs_idx(a, r, i)];
      vr = (float)fv.x * scr;
      vi = (float)fv.y * sci;
    } else {
      vr = (float)reinterpret_cast<const T*>(a.fs)[fs_idx(a, r, i)] * scr;
    }
    const cplx<T> u = loc[i];
    switch (a.w) {
#define SBD_SW(W) case W: spread_point_fixed<T, CPLX, W>(ire, iim, a.SG, a.PL, u, vr, vi, two_over_w, beta, lane); break;
      SBD_SW(4) SBD_SW(5) SBD_SW(6) SBD_SW(7) SBD_SW(8) SBD_SW(9) SBD_SW(10) SBD_SW(11) SBD_SW(12)
      SBD_SW(13) SBD_SW(14) SBD_SW(15) SBD_SW(16)
#undef SBD_SW
      default: break;
    }
  }
  __syncthreads();
  const float ir = 1.0f / scr, ii = 1.0f / sci;
  for (int k = threadIdx.x; k < SG2; k += blockDim.x) {
    if (CPLX) {
      out[2 * k] = (T)((float)ire[k] * ir);
      out[2 * k + 1] = (T)((float)iim[k] * ii);
    } else {
      out[k] = (T)((float)ire[k] * ir);
    }
  }
}

// FP64 plans in deterministic mode: the same scheme in 64-bit fixed point (ds_add_u64;
// per-tile scale 2^61 / (1.01 S), resolution S 2^-61, about 4e-19 S).  Integer sums do not
// depend on the order of the atomic updates, so the tile, and q, are bit-reproducible.
template <bool CPLX>
__global__ void __launch_bounds__(256) k_spread_fixed64(ApplyArgs a) {
  extern __shared__ unsigned char smem_raw[];
  unsigned long long* ire = reinterpret_cast<unsigned long long*>(smem_raw);
  unsigned long long* iim = ire + a.SG * a.SG;
  __shared__ double red[2][256 / 64];
  const int64_t t = blockIdx.x;
  const int r = blockIdx.y;
  const int SG2 = a.SG * a.SG;
  for (int k = threadIdx.x; k < SG2; k += blockDim.x) {
    ire[k] = 0ull;
    if (CPLX) iim[k] = 0ull;
  }
  const int32_t s = a.tile_start[t], e = a.tile_start[t + 1];
  const int cnt = e - s;
  const int R = (cnt + 63) / 64;
  double sr = 0.0, si = 0.0;
  for (int kk = threadIdx.x; kk < 64 * R; kk += blockDim.x) {
    const int p = (kk & 63) * R + (kk >> 6);
    if (p >= cnt) continue;
    const int32_t i = s + p;
    double fr, fi;
    load_f(a.f, a.in_dtype, (int64_t)r * a.n + (a.sorted_io ? i : a.perm[i]), fr, fi);
    if (CPLX) reinterpret_cast<double2*>(a.fs)[fs_idx(a, r, i)] = make_double2(fr, fi);
    else reinterpret_cast<double*>(a.fs)[fs_idx(a, r, i)] = fr;
    sr += fabs(fr);
    si += fabs(fi);
  }
  for (int off = 32; off > 0; off >>= 1) {
    sr += __shfl_down(sr, off, 64);
    si += __shfl_down(si, off, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    red[0][threadIdx.x >> 6] = sr;
    red[1][threadIdx.x >> 6] = si;
  }
  __syncthreads();
  double tr = 0.0, ti = 0.0;
  for (int k = 0; k < (int)(blockDim.x >> 6); ++k) {
    tr += red[0][k];
    ti += red[1][k];
  }
  double* out = reinterpret_cast<double*>(a.sub) + ((int64_t)r * a.ntiles + t) * (int64_t)SG2 * (CPLX ? 2 : 1);
  if (!(tr <= 1.0e300) || !(ti <= 1.0e300)) {
    // non-finite f: no fixed-point scale exists; the tile is written as NaN (see k_spread_fixed)
    for (int k = threadIdx.x; k < SG2 * (CPLX ? 2 : 1); k += blockDim.x) out[k] = __builtin_nan("");
    return;
  }
  const double scr = tr > 0.0 ? 2305843009213693952.0 / (1.01 * tr) : 1.0;
  const double sci = ti > 0.0 ? 2305843009213693952.0 / (1.01 * ti) : 1.0;
  const double2* loc = reinterpret_cast<const double2*>(a.loc);
  const double two_over_w = 2.0 / (double)a.w;
  const double beta = a.beta;
  const double halfw = 0.5 * (double)a.w;
  const int lane = threadIdx.x & 63;
  for (int kk = threadIdx.x; kk < 64 * R; kk += blockDim.x) {
    const int p = (kk & 63) * R + (kk >> 6);
    if (p >= cnt) continue;
    const int32_t i = s + p;
    double vr, vi = 0.0;
    if (CPLX) {
      const double2 fv = reinterpret_cast<const double2*>(a.fs)[fs_idx(a, r, i)];
      vr = fv.x * scr;
      vi = fv.y * sci;
    } else {
      vr = reinterpret_cast<const double*>(a.fs)[fs_idx(a, r, i)] * scr;
    }
    const double2 u = loc[i];
    const int jx0 = (int)floor(u.x - halfw) + 1;
    const int jy0 = (int)floor(u.y - halfw) + 1;
    double wx[16];
    for (int k = 0; k < a.w; ++k) wx[k] = es_kernel<double>((double)(jx0 + k) - u.x, two_over_w, beta);
    int b = lane % a.w;
    for (int jb = 0; jb < a.w; ++jb) {
      const double wyb = es_kernel<double>((double)(jy0 + b) - u.y, two_over_w, beta);
      const int rowoff = (jy0 + b + a.PL) * a.SG + jx0 + a.PL;
      const double vyr = vr * wyb, vyi = vi * wyb;
      for (int k = 0; k < a.w; ++k) {
        atomicAdd(&ire[rowoff + k], (unsigned long long)__double2ll_rn(vyr * wx[k]));
        if (CPLX) atomicAdd(&iim[rowoff + k], (unsigned long long)__double2ll_rn(vyi * wx[k]));
      }
      b = (b + 1 == a.w) ? 0 : b + 1;
    }
  }
  __syncthreads();
  const double ir = 1.0 / scr, ii = 1.0 / sci;
  for (int k = threadIdx.x; k < SG2; k += blockDim.x) {
    if (CPLX) {
      out[2 * k] = (double)(long long)ire[k] * ir;
      out[2 * k + 1] = (double)(long long)iim[k] * ii;
    } else {
      out[k] = (double)(long long)ire[k] * ir;
    }
  }
}

template <typename T>
__device__ __forceinline__ void two_sum(T a, T b, T& s, T& e) {
  s = a + b;
  T bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}

// Assemble FFT-grid row Y from the overlapping tile subgrids (at most 2 x 2 tiles
// cover a cell), summing the overlaps with a compensated (two-sum) reduction.
template <typename T, bool CPLX>
__global__ void k_gather_grid(ApplyArgs a) {
  const int64_t X = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t Y = blockIdx.y;
  const int r = blockIdx.z;
  if (X >= a.nx) return;
  const int Tt = a.T;
  const int64_t SG2 = (int64_t)a.SG * a.SG;
  T sr = 0, er = 0, si = 0, ei = 0;
  int64_t tyhi = Y / Tt, txhi = X / Tt;
  const T* sub = reinterpret_cast<const T*>(a.sub);
  for (int64_t ty = tyhi; ty >= 0 && ty >= tyhi - 1; --ty) {
    if (ty >= (a.ny - 2 * a.PL) / Tt) continue;
    int64_t ly = Y - ty * Tt;
    if (ly >= a.SG) continue;
    for (int64_t tx = txhi; tx >= 0 && tx >= txhi - 1; --tx) {
      if (tx >= a.ntx) continue;
      int64_t lx = X - tx * Tt;
      if (lx >= a.SG) continue;
      int64_t tile = ty * a.ntx + tx;
      int64_t off = (((int64_t)r * a.ntiles + tile) * SG2 + ly * a.SG + lx);
      if (CPLX) {
        T vr = sub[2 * off], vi = sub[2 * off + 1];
        T s1, e1;
        two_sum<T>(sr, vr, s1, e1); sr = s1; er += e1;
        two_sum<T>(si, vi, s1, e1); si = s1; ei += e1;
      } else {
        T v = sub[off];
        T s1, e1;
        two_sum<T>(sr, v, s1, e1); sr = s1; er += e1;
      }
    }
  }
  cplx<T>* g = reinterpret_cast<cplx<T>*>(a.grid) + (int64_t)r * a.My * a.Mx;
  g[Y * a.Mx + X] = mk<T>(sr + er, CPLX ? si + ei : T(0));
}

// Interpolate the convolved grid at the tile's points (NUFFT_+ side) and add the
// close correction rows of D (CSR), then write q in input order.
//
// The tile's grid window stays in LDS; points are handled in chunks of rows.  The
// far part is one point per thread.  The close part has three traversals (NearMode):
// the default flat one gives each thread runs of 8 consecutive CSR entries and adds
// row partial sums into the rows' LDS slots; the pipelined and plain ones give each
// CSR row to a group of 16 consecutive lanes (one DPP row) and form the row sums with
// DPP rotations.

// Sum of a double over the 16 lanes of a DPP row (every lane receives the sum):
// rotate-right by 8, 4, 2, 1 within the row and add (VALU data-parallel
// primitives; no LDS traffic).
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
  int2 x = *reinterpret_cast<int2*>(&v);
  int2 y;
  y.x = __builtin_amdgcn_update_dpp(0, x.x, CTRL, 0xF, 0xF, false);
  y.y = __builtin_amdgcn_update_dpp(0, x.y, CTRL, 0xF, 0xF, false);
  return *reinterpret_cast<double*>(&y);
}
template <int CTRL>
__device__ __forceinline__ float dpp_f(float v) {
  int x = __float_as_int(v);
  return __int_as_float(__builtin_amdgcn_update_dpp(0, x, CTRL, 0xF, 0xF, false));
}
__device__ __forceinline__ double row16_sum(double v) {
  v += dpp_d<0x128>(v);  // row_ror:8
  v += dpp_d<0x124>(v);  // row_ror:4
  v += dpp_d<0x122>(v);  // row_ror:2
  v += dpp_d<0x121>(v);  // row_ror:1
  return v;
}
__device__ __forceinline__ float row16_sum(float v) {
  v += dpp_f<0x128>(v);
  v += dpp_f<0x124>(v);
  v += dpp_f<0x122>(v);
  v += dpp_f<0x121>(v);
  return v;
}

// Far part at one point: sum over the W x W cells of phi(x_g - z) times the grid value
// (W a compile-time constant, so the taps are unrolled into LDS reads with immediate
// offsets).
template <typename T, bool CPLX, int W>
__device__ __forceinline__ void interp_point(const T* sre, const T* sim, int SG, int PL, cplx<T> u, T two_over_w,
                                             T beta, double& ar, double& ai) {
  const T halfw = T(0.5) * T(W);
  const int jx0 = (int)floor(u.x - halfw) + 1;
  const int jy0 = (int)floor(u.y - halfw) + 1;
  T wx[W];
#pragma unroll
  for (int m = 0; m < W; ++m) wx[m] = es_kernel<T>(T(jx0 + m) - u.x, two_over_w, beta);
  const int base = (jy0 + PL) * SG + jx0 + PL;
  T sr = 0, si = 0;
#pragma unroll
  for (int b = 0; b < W; ++b) {
    const T wyb = es_kernel<T>(T(jy0 + b) - u.y, two_over_w, beta);
    const T* rp = sre + base + b * SG;
    T rr = 0, ri = 0;
#pragma unroll
    for (int m = 0; m < W; ++m) rr += wx[m] * rp[m];
    if (CPLX) {
      const T* ip = sim + base + b * SG;
#pragma unroll
      for (int m = 0; m < W; ++m) ri += wx[m] * ip[m];
    }
    sr += wyb * rr;
    if (CPLX) si += wyb * ri;
  }
  ar = sr;
  ai = CPLX ? (double)si : 0.0;
}

// Far part at one point for a runtime kernel width w <= 16.
template <typename T, bool CPLX>
__device__ __forceinline__ void interp_point_rt(const T* sre, const T* sim, int SG, int PL, int w, cplx<T> u,
                                                T two_over_w, T beta, double& ar, double& ai) {
  const T halfw = T(0.5) * T(w);
  const int jx0 = (int)floor(u.x - halfw) + 1;
  const int jy0 = (int)floor(u.y - halfw) + 1;
  T wx[16];
  for (int m = 0; m < w; ++m) wx[m] = es_kernel<T>(T(jx0 + m) - u.x, two_over_w, beta);
  T sr = 0, si = 0;
  for (int b = 0; b < w; ++b) {
    const T wyb = es_kernel<T>(T(jy0 + b) - u.y, two_over_w, beta);
    const int rowoff = (jy0 + b + PL) * SG + jx0 + PL;
    T rr = 0, ri = 0;
    for (int m = 0; m < w; ++m) {
      rr += wx[m] * sre[rowoff + m];
      if (CPLX) ri += wx[m] * sim[rowoff + m];
    }
    sr += wyb * rr;
    if (CPLX) si += wyb * ri;
  }
  ar = sr;
  ai = CPLX ? (double)si : 0.0;
}

// Close-part traversal of k_interp_near.
enum NearMode { kNearPlain = 0, kNearPipelined = 1, kNearFlat = 2 };

template <typename T, bool CPLX, typename VT, int kRowsInFlight, int kInterpChunk, int MODE>
__global__ void __launch_bounds__(256) k_interp_near(ApplyArgs a) {
  // close-correction products accumulate in the precision of the stored D
  using AT = VT;
  extern __shared__ unsigned char smem_raw[];
  double* qre = reinterpret_cast<double*>(smem_raw);
  double* qim = qre + kInterpChunk;
  int32_t* roff = reinterpret_cast<int32_t*>(qim + kInterpChunk);
  T* sre = reinterpret_cast<T*>(roff + kInterpChunk + 4);
  T* sim = sre + a.SG * a.SG;
  // one workgroup per work unit: a run of at most kInterpChunk sorted points of one tile
  // (dense tiles are split so that units carry similar close-correction work)
  const int64_t unit = blockIdx.x;
  const int64_t t = a.unit_tile[unit];
  const int r = blockIdx.y;
  const int64_t tx = t % a.ntx, ty = t / a.ntx;
  const int SG2 = a.SG * a.SG;
  const bool far = (a.parts & 1) != 0;
  const bool near = (a.parts & 2) != 0 && !a.qnear;  // this kernel's own close traversal
  if (far) {
    const cplx<T>* g = reinterpret_cast<const cplx<T>*>(a.grid) + (int64_t)r * a.My * a.Mx;
    const T* gr = reinterpret_cast<const T*>(g);
    for (int k = threadIdx.x; k < SG2; k += blockDim.x) {
      int ly = k / a.SG, lx = k - ly * a.SG;
      int64_t Y = ty * a.T + ly, X = tx * a.T + lx;
      if (!CPLX && a.real_grid) {
        sre[k] = (Y < a.ny && X < a.nx) ? gr[Y * 2 * a.Mx + X] : T(0);
      } else {
        cplx<T> v = mk<T>(T(0), T(0));
        if (Y < a.ny && X < a.nx) v = g[Y * a.Mx + X];
        sre[k] = v.x;
        if (CPLX) sim[k] = v.y;
      }
    }
  }
  __syncthreads();
  const int32_t s = a.unit_start[unit], e = a.unit_start[unit + 1];
  const cplx<T>* loc = reinterpret_cast<const cplx<T>*>(a.tloc);
  const T two_over_w = T(2) / T(a.w);
  const T beta = (T)a.beta;
  const T halfw = T(0.5) * T(a.w);
  const int lane = threadIdx.x & 63;
  for (int32_t c0 = s; c0 < e; c0 += kInterpChunk) {
    const int cnt = min(kInterpChunk, e - c0);
    for (int p = threadIdx.x; p < cnt; p += blockDim.x) {
      double ar = 0.0, ai = 0.0;
      if (far) {
        const cplx<T> u = loc[c0 + p];
        if constexpr (sizeof(T) == 4) {
          switch (a.w) {
#define SBD_IW(W) case W: interp_point<T, CPLX, W>(sre, sim, a.SG, a.PL, u, two_over_w, beta, ar, ai); break;
            SBD_IW(4) SBD_IW(5) SBD_IW(6) SBD_IW(7) SBD_IW(8) SBD_IW(9) SBD_IW(10) SBD_IW(11) SBD_IW(12)
            SBD_IW(13) SBD_IW(14) SBD_IW(15) SBD_IW(16)
#undef SBD_IW
            default: break;
          }
        } else {
          // FP64: a runtime-width loop (unrolled FP64 exponentials for every width exceed
          // the register file)
          interp_point_rt<T, CPLX>(sre, sim, a.SG, a.PL, a.w, u, two_over_w, beta, ar, ai);
        }
      }
      if (a.qnear) {  // the close correction summed by k_near_multi
        if (CPLX) {
          const double2 v = reinterpret_cast<const double2*>(a.qnear)[(int64_t)r * a.nt + c0 + p];
          ar += v.x;
          ai += v.y;
        } else {
          ar += reinterpret_cast<const double*>(a.qnear)[(int64_t)r * a.nt + c0 + p];
        }
      }
      qre[p] = ar;
      if (CPLX) qim[p] = ai;
    }
    int64_t kbase = 0;
    if (near) {
      kbase = a.row_ptr[c0];
      for (int p = threadIdx.x; p <= cnt; p += blockDim.x) roff[p] = (int32_t)(a.row_ptr[c0 + p] - kbase);
    }
    __syncthreads();
    if (near) {
      if constexpr (MODE == kNearFlat) {
        // Flat traversal: the chunk's close entries are cut into runs of 8 consecutive
        // entries (aligned to 8 in the whole CSR, so whole runs load as 16-byte vectors);
        // a thread finds the row of its run's first entry by binary search in roff,
        // gathers the run's 8 source values at once, walks the run in order and adds
        // each row's partial sum into that row's LDS slot (FP64 LDS atomics) whenever
        // the row ends and at the end of the run.  Every lane carries entries whatever
        // the row lengths.
        const int64_t k0 = kbase, k1 = kbase + roff[cnt];
        const T* __restrict__ fsr = reinterpret_cast<const T*>(a.fs) + (int64_t)r * a.n * (CPLX ? 2 : 1);
        const int32_t* __restrict__ colg = a.col;
        const VT* __restrict__ valg = reinterpret_cast<const VT*>(a.val);
        for (int64_t run = (k0 >> 3) + threadIdx.x; run < ((k1 + 7) >> 3); run += blockDim.x) {
          const int64_t e0 = run << 3;
          int cl[8];
          VT vl[8];
          if (e0 >= k0 && e0 + 8 <= k1) {
            const int4* c4 = reinterpret_cast<const int4*>(colg + e0);
            const int4 ca = c4[0], cb = c4[1];
            cl[0] = ca.x; cl[1] = ca.y; cl[2] = ca.z; cl[3] = ca.w;
            cl[4] = cb.x; cl[5] = cb.y; cl[6] = cb.z; cl[7] = cb.w;
#pragma unroll
            for (int i = 0; i < 8; ++i) vl[i] = valg[e0 + i];
          } else {
#pragma unroll
            for (int i = 0; i < 8; ++i) {
              const bool ok = e0 + i >= k0 && e0 + i < k1;
              cl[i] = ok ? colg[e0 + i] : -1;
              vl[i] = ok ? valg[e0 + i] : VT(0);
            }
          }
          T fx[8], fy[8];
#pragma unroll
          for (int i = 0; i < 8; ++i) {
            fx[i] = T(0);
            fy[i] = T(0);
            if (cl[i] >= 0) {
              if (CPLX) {
                const cplx<T> fv = reinterpret_cast<const cplx<T>*>(fsr)[cl[i]];
                fx[i] = fv.x;
                fy[i] = fv.y;
              } else {
                fx[i] = fsr[cl[i]];
              }
            }
          }
          // row of the run's first entry inside the chunk: last p with roff[p] <= rel
          int rel = (int)((e0 > k0 ? e0 : k0) - kbase);
          int lo = 0, hi = cnt - 1;
          while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (roff[mid] <= rel) lo = mid;
            else hi = mid - 1;
          }
          int prow = lo;
          int bound = roff[prow + 1];
          AT accr = AT(0), acci = AT(0);
#pragma unroll
          for (int i = 0; i < 8; ++i) {
            if (cl[i] < 0) continue;
            while (rel >= bound) {
              atomicAdd(&qre[prow], (double)accr);
              if (CPLX) atomicAdd(&qim[prow], (double)acci);
              accr = AT(0);
              acci = AT(0);
              ++prow;
              bound = roff[prow + 1];
            }
            accr += vl[i] * (AT)fx[i];
            if (CPLX) acci += vl[i] * (AT)fy[i];
            ++rel;
          }
          atomicAdd(&qre[prow], (double)accr);
          if (CPLX) atomicAdd(&qim[prow], (double)acci);
        }
      } else if constexpr (MODE == kNearPipelined) {
        // 16-lane groups own rows; each group keeps kRowsInFlight rows' loads in flight, and
        // the first 16 entries of the next round's rows are loaded while this round's f
        // gathers are outstanding (software pipelining of the dependent loads).
        const int gl = threadIdx.x & 15;
        const int gid = threadIdx.x >> 4;
        const int ngroups = blockDim.x >> 4;
        const int step = ngroups * kRowsInFlight;
        const int32_t* __restrict__ colp = a.col + kbase;
        const VT* __restrict__ valp = reinterpret_cast<const VT*>(a.val) + kbase;
        const T* __restrict__ fsr = reinterpret_cast<const T*>(a.fs) + (int64_t)r * a.n * (CPLX ? 2 : 1);
        int c0r[kRowsInFlight], c1r[kRowsInFlight], cidx[kRowsInFlight];
        AT vv[kRowsInFlight];
        auto fetch = [&](int pb, int* b0, int* b1, int* ci, AT* va) {
#pragma unroll
          for (int u = 0; u < kRowsInFlight; ++u) {
            const int p = pb + gid + u * ngroups;
            b0[u] = p < cnt ? roff[p] : 0;
            b1[u] = p < cnt ? roff[p + 1] : 0;
            const int c = b0[u] + gl;
            const bool ok = c < b1[u];
            ci[u] = ok ? colp[c] : -1;
            va[u] = ok ? (AT)valp[c] : AT(0);
          }
        };
        fetch(0, c0r, c1r, cidx, vv);
        for (int pb = 0; pb < cnt; pb += step) {
          AT nr[kRowsInFlight], ni[kRowsInFlight];
          T fx[kRowsInFlight], fy[kRowsInFlight];
#pragma unroll
          for (int u = 0; u < kRowsInFlight; ++u) {
            fx[u] = T(0);
            fy[u] = T(0);
            if (cidx[u] >= 0) {
              if (CPLX) {
                cplx<T> fv = reinterpret_cast<const cplx<T>*>(fsr)[cidx[u]];
                fx[u] = fv.x;
                fy[u] = fv.y;
              } else {
                fx[u] = fsr[cidx[u]];
              }
            }
          }
          int n0[kRowsInFlight], n1[kRowsInFlight], ncid[kRowsInFlight];
          AT nvv[kRowsInFlight];
          const bool more = pb + step < cnt;
          if (more) fetch(pb + step, n0, n1, ncid, nvv);
          int maxlen = 0;
#pragma unroll
          for (int u = 0; u < kRowsInFlight; ++u) {
            nr[u] = vv[u] * (AT)fx[u];
            ni[u] = CPLX ? vv[u] * (AT)fy[u] : AT(0);
            maxlen = max(maxlen, c1r[u] - c0r[u]);
          }
          // rows longer than 16 entries: the remaining entries, not pipelined
          for (int off = gl + 16; off < maxlen; off += 16) {
            int ci2[kRowsInFlight];
            AT v2[kRowsInFlight];
#pragma unroll
            for (int u = 0; u < kRowsInFlight; ++u) {
              const int c = c0r[u] + off;
              const bool ok = c < c1r[u];
              ci2[u] = ok ? colp[c] : -1;
              v2[u] = ok ? (AT)valp[c] : AT(0);
            }
#pragma unroll
            for (int u = 0; u < kRowsInFlight; ++u) {
              if (ci2[u] >= 0) {
                if (CPLX) {
                  cplx<T> fv = reinterpret_cast<const cplx<T>*>(fsr)[ci2[u]];
                  nr[u] += v2[u] * (AT)fv.x;
                  ni[u] += v2[u] * (AT)fv.y;
                } else {
                  nr[u] += v2[u] * (AT)fsr[ci2[u]];
                }
              }
            }
          }
#pragma unroll
          for (int u = 0; u < kRowsInFlight; ++u) {
            nr[u] = row16_sum(nr[u]);
            if (CPLX) ni[u] = row16_sum(ni[u]);
            const int p = pb + gid + u * ngroups;
            if (gl == 0 && p < cnt) {
              qre[p] += (double)nr[u];
              if (CPLX) qim[p] += (double)ni[u];
            }
          }
          if (more) {
#pragma unroll
            for (int u = 0; u < kRowsInFlight; ++u) {
              c0r[u] = n0[u];
              c1r[u] = n1[u];
              cidx[u] = ncid[u];
              vv[u] = nvv[u];
            }
          }
        }
      } else {
        // 16-lane groups own rows; each group keeps kRowsInFlight rows' loads in flight.
        const int gl = threadIdx.x & 15;
        const int gid = threadIdx.x >> 4;
        const int ngroups = blockDim.x >> 4;
        const int32_t* __restrict__ colp = a.col + kbase;
        const VT* __restrict__ valp = reinterpret_cast<const VT*>(a.val) + kbase;
        for (int pb = 0; pb < cnt; pb += ngroups * kRowsInFlight) {
          int c0r[kRowsInFlight], c1r[kRowsInFlight];
          AT nr[kRowsInFlight], ni[kRowsInFlight];
          int maxlen = 0;
#pragma unroll
          for (int u = 0; u < kRowsInFlight; ++u) {
            int p = pb + gid + u * ngroups;
            c0r[u] = p < cnt ? roff[p] : 0;
            c1r[u] = p < cnt ? roff[p + 1] : 0;
            maxlen = max(maxlen, c1r[u] - c0r[u]);
            nr[u] = AT(0);
            ni[u] = AT(0);
          }
          for (int off = gl; off < maxlen; off += 16) {
            int cidx[kRowsInFlight];
            AT vv[kRowsInFlight];
#pragma unroll
            for (int u = 0; u < kRowsInFlight; ++u) {
              int c = c0r[u] + off;
              bool ok = c < c1r[u];
              cidx[u] = ok ? colp[c] : -1;
              vv[u] = ok ? (AT)valp[c] : AT(0);
            }
#pragma unroll
            for (int u = 0; u < kRowsInFlight; ++u) {
              if (cidx[u] >= 0) {
                if (CPLX) {
                  cplx<T> fv = reinterpret_cast<const cplx<T>*>(a.fs)[fs_idx(a, r, cidx[u])];
                  nr[u] += vv[u] * (AT)fv.x;
                  ni[u] += vv[u] * (AT)fv.y;
                } else {
                  nr[u] += vv[u] * (AT)reinterpret_cast<const T*>(a.fs)[fs_idx(a, r, cidx[u])];
                }
              }
            }
          }
#pragma unroll
          for (int u = 0; u < kRowsInFlight; ++u) {
            nr[u] = row16_sum(nr[u]);
            if (CPLX) ni[u] = row16_sum(ni[u]);
            int p = pb + gid + u * ngroups;
            if (gl == 0 && p < cnt) {
              qre[p] += (double)nr[u];
              if (CPLX) qim[p] += (double)ni[u];
            }
          }
        }
      }
    }
    __syncthreads();
    for (int p = threadIdx.x; p < cnt; p += blockDim.x) {
      double qr = qre[p], qi = CPLX ? qim[p] : 0.0;
      if (CPLX && (a.parts & 2) && a.self) {
        cplx<T> fv = reinterpret_cast<const cplx<T>*>(a.fs)[fs_idx(a, r, c0 + p)];
        qr -= a.self_im * (double)fv.y;
        qi += a.self_im * (double)fv.x;
      }
      store_q(a.q, a.in_dtype, (int64_t)r * a.nt + (a.sorted_io ? c0 + p : a.tperm[c0 + p]), qr, qi);
    }
    __syncthreads();
  }
}

__global__ void k_to_f32(const double* __restrict__ src, float* __restrict__ dst, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = (float)src[i];
}

inline int last_err() { return hipGetLastError() == hipSuccess ? 0 : -5; }

}  // namespace

template <typename T>
int launch_reorder(const void* src, void* dst, int64_t Mx, int64_t My, int64_t L1x, int64_t L2x, int64_t L1y,
                   int64_t L2y, int to_natural, hipStream_t st) {
  hipLaunchKernelGGL(k_reorder<T>, dim3((unsigned)ceil_div(Mx, kBlock), (unsigned)My), dim3(kBlock), 0, st,
                     (const cplx<T>*)src, (cplx<T>*)dst, Mx, My, L1x, L2x, L1y, L2y, to_natural);
  return last_err();
}
template int launch_reorder<float>(const void*, void*, int64_t, int64_t, int64_t, int64_t, int64_t, int64_t, int, hipStream_t);
template int launch_reorder<double>(const void*, void*, int64_t, int64_t, int64_t, int64_t, int64_t, int64_t, int, hipStream_t);

int launch_bbox_partials(const double* pts, int64_t n, double* partials, int nblocks, hipStream_t st) {
  hipLaunchKernelGGL(k_bbox, dim3(nblocks), dim3(kBlock), 0, st, pts, n, partials);
  return last_err();
}

int launch_radius_partials(const double* pts, int64_t n, double cx, double cy, double* partials, int nblocks,
                           hipStream_t st) {
  hipLaunchKernelGGL(k_radius, dim3(nblocks), dim3(kBlock), 0, st, pts, n, cx, cy, partials);
  return last_err();
}

int launch_keys(const double* pts, const Layout& L, int32_t* keys, int32_t* counts, int* bad, hipStream_t st) {
  KeyArgs a{L.x0, L.y0, L.inv_c, L.ncx, L.ncy, L.ntx, L.nsub};
  hipLaunchKernelGGL(k_keys, dim3((unsigned)ceil_div(L.n, kBlock)), dim3(kBlock), 0, st, pts, L.n, a, keys, counts, bad);
  return last_err();
}

int launch_scatter(const int32_t* keys, int64_t n, const int32_t* cell_start, int32_t* fill, int32_t* perm,
                   hipStream_t st) {
  hipLaunchKernelGGL(k_scatter, dim3((unsigned)ceil_div(n, kBlock)), dim3(kBlock), 0, st, keys, n, cell_start, fill, perm);
  return last_err();
}

int launch_sort_cells(const int32_t* cell_start, int64_t nkeys, int32_t* perm, hipStream_t st) {
  hipLaunchKernelGGL(k_sort_cells, dim3((unsigned)ceil_div(nkeys, kBlock)), dim3(kBlock), 0, st, cell_start, nkeys, perm);
  return last_err();
}

template <typename T>
int launch_gather_sorted(const double* pts, const int32_t* perm, const Layout& L, double2* xs,
                         typename cplx_of<T>::type* loc, int32_t* skeys, const int32_t* keys, hipStream_t st) {
  GatherArgs a{L.x0, L.y0, L.inv_h, L.T, L.nsub, L.ntx};
  hipLaunchKernelGGL(k_gather_sorted<T>, dim3((unsigned)ceil_div(L.n, kBlock)), dim3(kBlock), 0, st, pts, perm, L.n, a,
                     xs, loc, skeys, keys);
  return last_err();
}
template int launch_gather_sorted<float>(const double*, const int32_t*, const Layout&, double2*, float2*, int32_t*,
                                         const int32_t*, hipStream_t);
template int launch_gather_sorted<double>(const double*, const int32_t*, const Layout&, double2*, double2*, int32_t*,
                                          const int32_t*, hipStream_t);

int launch_near_count(const double2* xt, const int32_t* tkeys, int64_t nt, const double2* xs,
                      const int32_t* cell_start, const Layout& L, double d2max, int self, int32_t* counts, int* dup,
                      hipStream_t st) {
  NearArgs a{nt, L.nsub, L.ntx, L.ncx, L.ncy, d2max};
  hipLaunchKernelGGL(k_near_count_g, dim3((unsigned)ceil_div(nt * kNearGroup, 256)), dim3(256), 0, st, xt, tkeys, xs,
                     cell_start, a, self, counts, dup);
  return last_err();
}

int launch_near_fill(const double2* xt, const int32_t* tkeys, int64_t nt, const double2* xs,
                     const int32_t* cell_start, const Layout& L, double d2max, int self, const int64_t* row_ptr,
                     int32_t* col, double* val, const double* chebA, const double* chebB, int deg, double U,
                     double self_re, int in_r, hipStream_t st) {
  NearArgs a{nt, L.nsub, L.ntx, L.ncx, L.ncy, d2max};
  FillArgs f{chebA, chebB, deg, U, self_re, in_r};
  hipLaunchKernelGGL(k_near_fill_g, dim3((unsigned)ceil_div(nt * kNearGroup, 256)), dim3(256), 0, st, xt, tkeys, xs,
                     cell_start, a, self, row_ptr, col, val, f);
  return last_err();
}


int launch_node_gather(const NodeSpreadArgs& a, int ncirc, hipStream_t st) {
  if (a.wt > 16) return -1;
  dim3 grid((unsigned)ceil_div(a.Kx, kNodeTile), (unsigned)ceil_div(a.Ky, kNodeTile));
  hipLaunchKernelGGL(k_node_gather, grid, dim3(kBlock), 0, st, a, ncirc);
  return last_err();
}

int launch_embed_symbol(const double2* fine, int64_t Kx, int64_t Ky, int64_t sx, int64_t sy, const double* invpsix,
                        const double* invpsiy, int64_t nx, int64_t ny, double2* emb, int64_t Mx, int64_t My,
                        hipStream_t st) {
  hipLaunchKernelGGL(k_embed, dim3((unsigned)ceil_div(Mx, kBlock), (unsigned)My), dim3(kBlock), 0, st, fine, Kx, Ky,
                     sx, sy, invpsix, invpsiy, nx, ny, emb, Mx, My);
  return last_err();
}

template <typename T>
int launch_store_symbol(const double2* emb, const SymbolRemap& r, double scale, int complex_out, void* out,
                        hipStream_t st) {
  hipLaunchKernelGGL(k_store_symbol<T>, dim3((unsigned)ceil_div(r.Mx, kBlock), (unsigned)r.My), dim3(kBlock), 0, st, emb,
                     r, scale, complex_out, out);
  return last_err();
}
template int launch_store_symbol<float>(const double2*, const SymbolRemap&, double, int, void*, hipStream_t);
template int launch_store_symbol<double>(const double2*, const SymbolRemap&, double, int, void*, hipStream_t);

template <typename T>
int launch_spread(const ApplyArgs& a, hipStream_t st) {
  if (a.w > 16) return -1;
  // accumulators: 32-bit fixed point (FP32 plans), FP64 or 64-bit fixed point (FP64 plans)
  const size_t lds = (size_t)a.SG * a.SG * (sizeof(T) == 4 ? 4 : 8) * (a.cplx_data ? 2 : 1);
  dim3 grid((unsigned)a.ntiles, (unsigned)a.nrhs);
  void (*kfn)(ApplyArgs);
  if (sizeof(T) == 4) kfn = a.cplx_data ? k_spread_fixed<T, true> : k_spread_fixed<T, false>;
  else if (a.deterministic) kfn = a.cplx_data ? k_spread_fixed64<true> : k_spread_fixed64<false>;
  else kfn = a.cplx_data ? k_spread<T, true> : k_spread<T, false>;
  if (lds > 65536) (void)hipFuncSetAttribute((const void*)kfn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  hipLaunchKernelGGL(kfn, grid, dim3(256), lds, st, a);
  int rc = last_err();
  {
    double er = sizeof(T), cp = a.cplx_data ? 2.0 : 1.0;
    double fin = (a.in_dtype == 0 ? 8.0 : a.in_dtype == 1 ? 4.0 : a.in_dtype == 2 ? 16.0 : 8.0);
    double b = (double)a.nrhs * ((double)a.n * (fin + er * cp) + (double)a.ntiles * a.SG * a.SG * er * cp) +
               (double)a.n * (4.0 + 2.0 * er);
    mark_launch("spread", st, b);
  }
  return rc;
}

template <typename T>
int launch_gather_grid(const ApplyArgs& a, hipStream_t st) {
  dim3 grid((unsigned)ceil_div(a.nx, kBlock), (unsigned)a.ny, (unsigned)a.nrhs);
  if (a.cplx_data) hipLaunchKernelGGL((k_gather_grid<T, true>), grid, dim3(kBlock), 0, st, a);
  else hipLaunchKernelGGL((k_gather_grid<T, false>), grid, dim3(kBlock), 0, st, a);
  int rc = last_err();
  {
    double er = sizeof(T), cp = a.cplx_data ? 2.0 : 1.0;
    double b = (double)a.nrhs * ((double)a.ntiles * a.SG * a.SG * er * cp + (double)a.nx * a.ny * 2.0 * er);
    mark_launch("grid_assembly", st, b);
  }
  return rc;
}

template <typename T>
int launch_interp_near(const ApplyArgs& a, hipStream_t st) {
  constexpr int chunk = kUnitPoints;
  size_t lds = (size_t)a.SG * a.SG * sizeof(T) * (a.cplx_data ? 2 : 1) + (size_t)kUnitPoints * 20 + 16;
  if (a.nunits <= 0) return 0;
  dim3 grid((unsigned)a.nunits, (unsigned)a.nrhs);
  // the flat traversal for every row length (measured at N = 1e7 uniform, about 11
  // entries per row: 0.42 ms against 0.52 ms pipelined and 0.59 ms plain; curves with
  // about 165 entries per row, 16 right-hand sides: 1.36 ms against 1.56 ms plain).
  // SBD_NEAR_MODE = 0 / 1 / 2 forces the plain, pipelined or flat traversal.
  const char* near_env = getenv("SBD_NEAR_MODE");  // read per launch, so a process can switch
  const int forced = near_env ? atoi(near_env) : -1;
  int mode = (forced >= 0 && forced <= 2) ? forced : kNearFlat;
  // the flat traversal meets row partial sums in LDS float atomics (order-dependent);
  // deterministic plans take the pipelined one, where one lane writes each row sum
  if (a.deterministic && mode == kNearFlat) mode = kNearPipelined;
  void (*kfn)(ApplyArgs);
#define SBD_IK(VT, M) (a.cplx_data ? k_interp_near<T, true, VT, 4, chunk, M> : k_interp_near<T, false, VT, 4, chunk, M>)
  if (a.val_f32)
    kfn = mode == kNearFlat ? SBD_IK(float, kNearFlat) : mode == kNearPipelined ? SBD_IK(float, kNearPipelined)
                                                                                  : SBD_IK(float, kNearPlain);
  else
    kfn = mode == kNearFlat ? SBD_IK(double, kNearFlat) : mode == kNearPipelined ? SBD_IK(double, kNearPipelined)
                                                                                   : SBD_IK(double, kNearPlain);
#undef SBD_IK
  if (lds > 65536) (void)hipFuncSetAttribute((const void*)kfn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  hipLaunchKernelGGL(kfn, grid, dim3(256), lds, st, a);
  int rc = last_err();
  {
    double er = sizeof(T), cp = a.cplx_data ? 2.0 : 1.0;
    double fout = (a.in_dtype == 0 ? 8.0 : a.in_dtype == 1 ? 4.0 : a.in_dtype == 2 ? 16.0 : 8.0);
    // targets' permutation and q
    double b = (double)a.nt * 4.0 + (double)a.nrhs * (double)a.nt * fout;
    // far part: targets' tile-local positions, the convolved grid
    if (a.parts & 1)
      b += (double)a.nt * 2.0 * er + (double)a.nrhs * (double)a.nx * a.ny * (a.real_grid && !a.cplx_data ? 1.0 : 2.0) * er;
    // close part: row pointers, columns and entries of D, the sorted f copy (or the sums
    // of k_near_multi)
    if ((a.parts & 2) && !a.qnear)
      b += (double)a.nt * 8.0 + (double)a.nnz * (a.val_f32 ? 8.0 : 12.0) + (double)a.nrhs * (double)a.n * er * cp;
    else if (a.parts & 2)
      b += (double)a.nrhs * (double)a.nt * 8.0 * cp;
    mark_launch("interp_near", st, b);
  }
  return rc;
}

int launch_to_f32(const double* src, float* dst, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_to_f32, dim3(2048), dim3(kBlock), 0, st, src, dst, n);
  return last_err();
}

template int launch_spread<float>(const ApplyArgs&, hipStream_t);
template int launch_spread<double>(const ApplyArgs&, hipStream_t);
template int launch_gather_grid<float>(const ApplyArgs&, hipStream_t);
template int launch_gather_grid<double>(const ApplyArgs&, hipStream_t);
template <typename T, bool CPLX, typename VT>
__global__ void __launch_bounds__(256) k_near_multi(ApplyArgs a, int rpad) {
  const int r = threadIdx.x & (rpad - 1);
  const int64_t row = (int64_t)blockIdx.x * (blockDim.x / rpad) + threadIdx.x / rpad;
  if (row >= a.nt || r >= a.nrhs) return;
  const VT* __restrict__ val = reinterpret_cast<const VT*>(a.val);
  const int64_t k1 = a.row_ptr[row + 1];
  double sr = 0.0, si = 0.0;
  int64_t k = a.row_ptr[row];
  // eight entries per step: their column and value loads, then their f gathers, are all in
  // flight together (the sums keep one fixed order per (row, r))
  constexpr int U = 8;
  for (; k + U <= k1; k += U) {
    int32_t c[U];
    double v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      c[u] = a.col[k + u];
      v[u] = (double)val[k + u];
    }
    if (CPLX) {
      cplx<T> f[U];
#pragma unroll
      for (int u = 0; u < U; ++u) f[u] = reinterpret_cast<const cplx<T>*>(a.fs)[(int64_t)c[u] * a.nrhs + r];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        sr += v[u] * (double)f[u].x;
        si += v[u] * (double)f[u].y;
      }
    } else {
      T f[U];
#pragma unroll
      for (int u = 0; u < U; ++u) f[u] = reinterpret_cast<const T*>(a.fs)[(int64_t)c[u] * a.nrhs + r];
#pragma unroll
      for (int u = 0; u < U; ++u) sr += v[u] * (double)f[u];
    }
  }
  for (; k < k1; ++k) {
    const int32_t c = a.col[k];
    const double v = (double)val[k];
    if (CPLX) {
      const cplx<T> f = reinterpret_cast<const cplx<T>*>(a.fs)[(int64_t)c * a.nrhs + r];
      sr += v * (double)f.x;
      si += v * (double)f.y;
    } else {
      sr += v * (double)reinterpret_cast<const T*>(a.fs)[(int64_t)c * a.nrhs + r];
    }
  }
  if (CPLX) reinterpret_cast<double2*>(a.qnear)[(int64_t)r * a.nt + row] = make_double2(sr, si);
  else reinterpret_cast<double*>(a.qnear)[(int64_t)r * a.nt + row] = sr;
}

template <typename T>
int launch_near_multi(const ApplyArgs& a, hipStream_t st) {
  if (!a.qnear || !a.fs_inter || a.nrhs < 2 || a.nrhs > 64) return -1;
  int rpad = 1;
  while (rpad < a.nrhs) rpad *= 2;
  const int64_t rows_per_block = kBlock / rpad;
  dim3 grid((unsigned)ceil_div(a.nt, rows_per_block));
  void (*kfn)(ApplyArgs, int);
  if (a.val_f32) kfn = a.cplx_data ? k_near_multi<T, true, float> : k_near_multi<T, false, float>;
  else kfn = a.cplx_data ? k_near_multi<T, true, double> : k_near_multi<T, false, double>;
  hipLaunchKernelGGL(kfn, grid, dim3(kBlock), 0, st, a, rpad);
  int rc = last_err();
  {
    const double er = sizeof(T), cp = a.cplx_data ? 2.0 : 1.0;
    mark_launch("near_multi", st,
                (double)a.nt * 8.0 + (double)a.nnz * (a.val_f32 ? 8.0 : 12.0) +
                    (double)a.nrhs * ((double)a.n * er * cp + (double)a.nt * 8.0 * cp));
  }
  return rc;
}
template int launch_near_multi<float>(const ApplyArgs&, hipStream_t);
template int launch_near_multi<double>(const ApplyArgs&, hipStream_t);

template int launch_interp_near<float>(const ApplyArgs&, hipStream_t);
template int launch_interp_near<double>(const ApplyArgs&, hipStream_t);

}  // namespace sbd
