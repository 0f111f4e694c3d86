// Close-correction entries by the pair-difference NUFFT (gfx950).
//
// Section 1 (eq. "defD") defines D_kl = G(z_k - z_l) - sum_nu omega_hat_nu exp(i (z_k - z_l) . xi_nu)
// on the close pairs and observes that the sum is a non-uniform Fourier transform from
// the circle nodes xi to the pair differences y = z_k - z_l; Section 6.1 (eq.
// "Complex:assemble") prices it as one NUFFT.  Here it is a type-3 transform in two FP64
// steps:
//  1. every node is spread with the ES kernel phi (width w cells) onto a G x G grid of
//     spacing h in frequency:  b_j = sum_nu c_nu phi(j_x - xi_x / h) phi(j_y - xi_y / h);
//  2. at each pair difference y,
//        F(y) = [sum_j b_j exp(i h y . j)] / (phi_hat(h y_x) phi_hat(h y_y)).
// By Poisson summation, sum_j phi(v - j) exp(i t j) = exp(i t v) phi_hat(t) plus aliases
// phi_hat(2 pi m - t), m != 0; with h = pi / (2 delta_min) every pair has |t| <= pi / 2
// (twofold oversampling), where the aliases stay below the kernel's tabulated error.
// Nodes lie in |xi| <= S, so the grid needs about 2 (2 S delta_min / pi + w / 2) cells per
// axis: a few dozen for the apply's circles, whatever N is.
//
// Step 1 is a contraction over the nodes with a G x G result: workgroups take chunks of
// nodes, tabulate each node's w weights per axis in LDS, and every wave accumulates its
// share of the chunk over the whole grid in registers (a lane holds a G/8 x G/8 block of
// cells); each wave writes one partial grid, summed afterwards in a fixed order (no
// atomics: the entries are bit-reproducible).  Step 2 runs one pair per lane; the grid
// is read with wave-uniform addresses, and the plane waves advance by rotation.
#include <algorithm>
#include <cmath>

#include "devmath.h"
#include "kernels.h"

namespace sbd {

namespace {

constexpr int kPdChunk = 32;       // nodes per LDS chunk
constexpr int kPdMaxBlocks = 512;  // spread workgroups (4 partial grids each)

int hip_rc() { return hipGetLastError() == hipSuccess ? 0 : -5; }

template <int NB>  // grid edge G = 8 NB
__global__ void __launch_bounds__(256) k_pd_spread(PdArgs a, double2* partials) {
  constexpr int G = 8 * NB;
  __shared__ double px[kPdChunk][G];   // phi(j_x - v_x) of each node of the chunk
  __shared__ double2 py[kPdChunk][G];  // c phi(j_y - v_y)
  __shared__ double nvx[kPdChunk], nvy[kPdChunk];
  __shared__ double2 nc[kPdChunk];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int cx = lane & 7, cy = lane >> 3;  // cells (cx + 8 u, cy + 8 v)
  double2 acc[NB][NB];
  for (int v = 0; v < NB; ++v)
    for (int u = 0; u < NB; ++u) acc[v][u] = make_double2(0.0, 0.0);
  const double inv_h = 1.0 / a.h, half = 0.5 * G, tw = 2.0 / a.w, hw = 0.5 * a.w;
  for (int64_t base = (int64_t)blockIdx.x * kPdChunk; base < a.nnodes; base += (int64_t)gridDim.x * kPdChunk) {
    for (int t = threadIdx.x; t < kPdChunk * G; t += blockDim.x) {
      (&px[0][0])[t] = 0.0;
      (&py[0][0])[t] = make_double2(0.0, 0.0);
    }
    if (threadIdx.x < kPdChunk) {
      const int64_t nu = base + threadIdx.x;
      double vx = half, vy = half;
      double2 c = make_double2(0.0, 0.0);  // past the last node: no contribution
      if (nu < a.nnodes) {
        int lo = 0, hi = a.ncirc;  // circle p with node_start[p] <= nu < node_start[p + 1]
        while (hi - lo > 1) {
          const int mid = (lo + hi) >> 1;
          if (a.node_start[mid] <= nu) lo = mid; else hi = mid;
        }
        const int64_t M = a.node_start[lo + 1] - a.node_start[lo];
        const int64_t m = nu - a.node_start[lo];
        double sn, cs;
        sincospi(2.0 * (double)m / (double)M, &sn, &cs);
        const double R = a.radius[lo];
        vx = R * cs * inv_h + half;
        vy = R * sn * inv_h + half;
        c = a.weight[lo];
      }
      nvx[threadIdx.x] = vx;
      nvy[threadIdx.x] = vy;
      nc[threadIdx.x] = c;
    }
    __syncthreads();
    for (int t = threadIdx.x; t < kPdChunk * a.w; t += blockDim.x) {
      const int k = t / a.w, s = t - k * a.w;
      const double vx = nvx[k], vy = nvy[k];
      const int jx = (int)floor(vx - hw) + 1 + s, jy = (int)floor(vy - hw) + 1 + s;
      if (jx >= 0 && jx < G) px[k][jx] = es_kernel<double>((double)jx - vx, tw, a.beta);
      if (jy >= 0 && jy < G) {
        const double f = es_kernel<double>((double)jy - vy, tw, a.beta);
        const double2 c = nc[k];
        py[k][jy] = make_double2(c.x * f, c.y * f);
      }
    }
    __syncthreads();
    for (int k = wave; k < kPdChunk; k += 4) {
      double xv[NB];
      double2 yv[NB];
      for (int u = 0; u < NB; ++u) xv[u] = px[k][cx + 8 * u];
      for (int v = 0; v < NB; ++v) yv[v] = py[k][cy + 8 * v];
      for (int v = 0; v < NB; ++v)
        for (int u = 0; u < NB; ++u) {
          acc[v][u].x += xv[u] * yv[v].x;
          acc[v][u].y += xv[u] * yv[v].y;
        }
    }
    __syncthreads();
  }
  double2* out = partials + ((int64_t)blockIdx.x * 4 + wave) * G * G;
  for (int v = 0; v < NB; ++v)
    for (int u = 0; u < NB; ++u) out[(cy + 8 * v) * G + cx + 8 * u] = acc[v][u];
}

// one workgroup per cell: strided partial sums, then a fixed LDS tree
__global__ void __launch_bounds__(256) k_pd_reduce(const double2* __restrict__ partials, int64_t nparts, int G,
                                                   double2* b) {
  __shared__ double sr[256], si[256];
  const int64_t c = blockIdx.x;
  const int64_t cells = (int64_t)G * G;
  double r = 0.0, i = 0.0;
  for (int64_t p = threadIdx.x; p < nparts; p += blockDim.x) {
    const double2 v = partials[p * cells + c];
    r += v.x;
    i += v.y;
  }
  sr[threadIdx.x] = r;
  si[threadIdx.x] = i;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      sr[threadIdx.x] += sr[threadIdx.x + s];
      si[threadIdx.x] += si[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) b[c] = make_double2(sr[0], si[0]);
}

__global__ void __launch_bounds__(256) k_pd_eval(PdArgs a, const double2* __restrict__ b,
                                                 const double* __restrict__ phihat, int deg, double tmax,
                                                 const double2* __restrict__ xt, const double2* __restrict__ xs,
                                                 const int64_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
                                                 int64_t nrows, int64_t nnz, int self, int kind, double wavenumber,
                                                 double* val) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= nnz) return;
  int64_t lo = 0, hi = nrows;  // row: row_ptr[lo] <= e < row_ptr[lo + 1]
  while (hi - lo > 1) {
    const int64_t mid = (lo + hi) >> 1;
    if (row_ptr[mid] <= e) lo = mid; else hi = mid;
  }
  const int32_t j = col[e];
  const double2 p = xt[lo], q = xs[j];
  const double yx = p.x - q.x, yy = p.y - q.y;
  const double tx = a.h * yx, ty = a.h * yy;
  double sx, cx, sy, cy, s0x, c0x, s0y, c0y;
  sincos(tx, &sx, &cx);
  sincos(ty, &sy, &cy);
  sincos(-(double)a.J * tx, &s0x, &c0x);
  sincos(-(double)a.J * ty, &s0y, &c0y);
  const int half = a.G / 2;
  // Re sum_j b_j exp(i (tx jx + ty jy)) over |jx|, |jy| <= J
  double fr = 0.0;
  double eyr = c0y, eyi = s0y;
  for (int jy = -a.J; jy <= a.J; ++jy) {
    const double2* row = b + (int64_t)(jy + half) * a.G + (half - a.J);
    double exr = c0x, exi = s0x, rr = 0.0, ri = 0.0;
    for (int jx = 0; jx <= 2 * a.J; ++jx) {
      const double2 v = row[jx];
      rr += v.x * exr - v.y * exi;
      ri += v.x * exi + v.y * exr;
      const double t = exr * cx - exi * sx;
      exi = exr * sx + exi * cx;
      exr = t;
    }
    fr += rr * eyr - ri * eyi;
    const double t = eyr * cy - eyi * sy;
    eyi = eyr * sy + eyi * cy;
    eyr = t;
  }
  const double phx = cheb_eval(phihat, deg, 2.0 * fabs(tx) / tmax - 1.0);
  const double phy = cheb_eval(phihat, deg, 2.0 * fabs(ty) / tmax - 1.0);
  double g = 0.0;  // the diagonal of a single point set has no G term
  if (!(self && j == lo)) {
    const double d2 = yx * yx + yy * yy;
    g = kind == 0 ? -0.079577471545947667884 * log(d2) : -0.25 * y0(wavenumber * sqrt(d2));
  }
  val[e] = g - fr / (phx * phy);
}

}  // namespace

int64_t pd_partials(int64_t nnodes) {
  const int64_t chunks = std::max<int64_t>(1, (nnodes + kPdChunk - 1) / kPdChunk);
  return 4 * std::min<int64_t>(kPdMaxBlocks, chunks);
}

int launch_pd_spread(const PdArgs& a, double2* partials, hipStream_t st) {
  if (a.G < 8 || a.G > kPdMaxGrid || a.G % 8 || a.w < 2 || a.w > 16 || a.J < 0 || 2 * a.J + 2 > a.G ||
      a.ncirc < 1 || a.nnodes < 1)
    return -1;
  const dim3 grid((unsigned)(pd_partials(a.nnodes) / 4));
  switch (a.G / 8) {
    case 1: hipLaunchKernelGGL(k_pd_spread<1>, grid, dim3(256), 0, st, a, partials); break;
    case 2: hipLaunchKernelGGL(k_pd_spread<2>, grid, dim3(256), 0, st, a, partials); break;
    case 3: hipLaunchKernelGGL(k_pd_spread<3>, grid, dim3(256), 0, st, a, partials); break;
    case 4: hipLaunchKernelGGL(k_pd_spread<4>, grid, dim3(256), 0, st, a, partials); break;
    case 5: hipLaunchKernelGGL(k_pd_spread<5>, grid, dim3(256), 0, st, a, partials); break;
    default: hipLaunchKernelGGL(k_pd_spread<6>, grid, dim3(256), 0, st, a, partials); break;
  }
  return hip_rc();
}

int launch_pd_reduce(const double2* partials, int64_t nparts, int G, double2* b, hipStream_t st) {
  if (G < 8 || G > kPdMaxGrid || nparts < 1) return -1;
  hipLaunchKernelGGL(k_pd_reduce, dim3((unsigned)(G * G)), dim3(256), 0, st, partials, nparts, G, b);
  return hip_rc();
}

int launch_pd_eval(const PdArgs& a, const double2* b, const double* phihat, int deg, double tmax, const double2* xt,
                   const double2* xs, const int64_t* row_ptr, const int32_t* col, int64_t nrows, int64_t nnz,
                   int self, int kind, double wavenumber, double* val, hipStream_t st) {
  if (nnz <= 0) return 0;
  if (a.G < 8 || a.G > kPdMaxGrid || 2 * a.J + 2 > a.G || nrows < 1 || (kind != 0 && kind != 1)) return -1;
  hipLaunchKernelGGL(k_pd_eval, dim3((unsigned)((nnz + 255) / 256)), dim3(256), 0, st, a, b, phihat, deg, tmax, xt,
                     xs, row_ptr, col, nrows, nnz, self, kind, wavenumber, val);
  return hip_rc();
}

}  // namespace sbd
