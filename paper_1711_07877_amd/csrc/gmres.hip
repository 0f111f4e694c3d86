// Restarted GMRES on the SBD operator (the iterative-solver use of the fast
// matvec that the Introduction motivates: integral equations whose dense
// matrix is G(z_k - z_l) times quadrature weights).
//
// Operator:  (A v)_k = sum_{l != k} G(z_k - z_l) w_l v_l + d_k v_k,
// i.e. sbd_apply of (w o v) plus a diagonal.  Arnoldi uses classical
// Gram-Schmidt applied twice (two projections per step, both done by
// device kernels), Givens rotations run on the host on the small Hessenberg
// column read back once per step.  All vectors are FP64 device arrays.
//
// One Arnoldi step (operator application, both projections, the new basis vector's
// norm and scaling) is captured once per solve as a HIP graph and replayed for every
// step: the step index j lives in device memory, so the captured kernels read it there
// (basis vector V[j] in, V[j + 1] out, j + 1 projections) and the last node increments
// it.  The host then reads back the step's Hessenberg column.
//
// The solve runs in the plan's sorted point order: b, the weights, the diagonal and the
// initial x are gathered through the plan's permutation once, every operator application
// reads and writes sorted vectors (SBD_IO_SORTED: no scattered accesses), and x is
// scattered back at the end.  Inner products and norms do not depend on the order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "../../include/sbd.h"
#include "common.h"

namespace sbd {
namespace {

constexpr int kThreads = 256;
constexpr int kMaxRestart = 64;

__device__ __forceinline__ double block_sum(double v, double* sh) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int k = 0; k < (int)(blockDim.x >> 6); ++k) t += sh[k];
  return t;
}

// part[i * nb + bx] = sum over this block's slice of V[i][k] * w[k], i = blockIdx.y.
__global__ void __launch_bounds__(kThreads) k_dot_partials(const double* __restrict__ V, int64_t ldv,
                                                            const double* __restrict__ w, int64_t n,
                                                            double* __restrict__ part) {
  __shared__ double sh[kThreads / 64];
  const double* v = V + (int64_t)blockIdx.y * ldv;
  double acc = 0.0;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x)
    acc += v[k] * w[k];
  double t = block_sum(acc, sh);
  if (threadIdx.x == 0) part[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = t;
}

// out[i] = sum_b part[i * nb + b] in a fixed order (deterministic), i = blockIdx.x.
__global__ void __launch_bounds__(kThreads) k_reduce_partials(const double* __restrict__ part, int nb,
                                                               double* __restrict__ out) {
  __shared__ double sh[kThreads / 64];
  double acc = 0.0;
  for (int b = threadIdx.x; b < nb; b += blockDim.x) acc += part[(int64_t)blockIdx.x * nb + b];
  double t = block_sum(acc, sh);
  if (threadIdx.x == 0) out[blockIdx.x] = t;
}

// w[k] += sign * sum_{i < cnt} h[i] * V[i][k]
__global__ void __launch_bounds__(kThreads) k_gemv_acc(double* __restrict__ w, const double* __restrict__ V,
                                                        int64_t ldv, int64_t n, const double* __restrict__ h,
                                                        int cnt, double sign) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  double acc = 0.0;
  for (int i = 0; i < cnt; ++i) acc += h[i] * V[(int64_t)i * ldv + k];
  w[k] += sign * acc;
}

// u = wts o v (wts NULL: copy)
__global__ void __launch_bounds__(kThreads) k_weight(double* __restrict__ u, const double* __restrict__ wts,
                                                      const double* __restrict__ v, int64_t n) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  u[k] = wts ? wts[k] * v[k] : v[k];
}

// out[i] = in[perm[i]]  (user order -> sorted order)
__global__ void __launch_bounds__(kThreads) k_gather_perm(double* __restrict__ out, const double* __restrict__ in,
                                                           const int32_t* __restrict__ perm, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = in[perm[i]];
}

// out[perm[i]] = in[i]  (sorted order -> user order)
__global__ void __launch_bounds__(kThreads) k_scatter_perm(double* __restrict__ out, const double* __restrict__ in,
                                                            const int32_t* __restrict__ perm, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[perm[i]] = in[i];
}

// y = sign * (y + d o v) + add   (d, add may be NULL)
__global__ void __launch_bounds__(kThreads) k_finish_op(double* __restrict__ y, const double* __restrict__ d,
                                                         const double* __restrict__ v, double sign,
                                                         const double* __restrict__ add, int64_t n) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  double t = y[k];
  if (d) t += d[k] * v[k];
  t *= sign;
  if (add) t += add[k];
  y[k] = t;
}

__global__ void __launch_bounds__(kThreads) k_scale(double* dst, const double* src,
                                                     double s, int64_t n) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) dst[k] = src[k] * s;
}

// ---- step kernels reading the step index j from device memory (graph-replayed)

// u = wts o V[j]
__global__ void __launch_bounds__(kThreads) k_weight_j(double* __restrict__ u, const double* __restrict__ wts,
                                                        const double* __restrict__ V, const int* __restrict__ jp,
                                                        int64_t n) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const double v = V[(int64_t)(*jp) * n + k];
  u[k] = wts ? wts[k] * v : v;
}

// w += d o V[j]
__global__ void __launch_bounds__(kThreads) k_diag_j(double* __restrict__ w, const double* __restrict__ d,
                                                      const double* __restrict__ V, const int* __restrict__ jp,
                                                      int64_t n) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  w[k] += d[k] * V[(int64_t)(*jp) * n + k];
}

// part[i * nb + bx] = slice sum of V[i] . w for i <= j (blocks with i > j return)
__global__ void __launch_bounds__(kThreads) k_dot_partials_j(const double* __restrict__ V, int64_t ldv,
                                                              const double* __restrict__ w, int64_t n,
                                                              const int* __restrict__ jp, double* __restrict__ part) {
  if ((int)blockIdx.y > *jp) return;
  __shared__ double sh[kThreads / 64];
  const double* v = V + (int64_t)blockIdx.y * ldv;
  double acc = 0.0;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x)
    acc += v[k] * w[k];
  double t = block_sum(acc, sh);
  if (threadIdx.x == 0) part[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = t;
}

__global__ void __launch_bounds__(kThreads) k_reduce_partials_j(const double* __restrict__ part, int nb,
                                                                 const int* __restrict__ jp, double* __restrict__ out) {
  if ((int)blockIdx.x > *jp) return;
  __shared__ double sh[kThreads / 64];
  double acc = 0.0;
  for (int b = threadIdx.x; b < nb; b += blockDim.x) acc += part[(int64_t)blockIdx.x * nb + b];
  double t = block_sum(acc, sh);
  if (threadIdx.x == 0) out[blockIdx.x] = t;
}

// w -= sum_{i <= j} h[i] V[i]
__global__ void __launch_bounds__(kThreads) k_gemv_j(double* __restrict__ w, const double* __restrict__ V,
                                                      int64_t n, const double* __restrict__ h,
                                                      const int* __restrict__ jp) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int cnt = *jp + 1;
  double acc = 0.0;
  for (int i = 0; i < cnt; ++i) acc += h[i] * V[(int64_t)i * n + k];
  w[k] -= acc;
}

// V[j + 1] = w / sqrt(hn) (hn > 0; else w unscaled: the host stops on a zero norm)
__global__ void __launch_bounds__(kThreads) k_store_next_j(double* __restrict__ V, const double* __restrict__ w,
                                                            const double* __restrict__ hn, const int* __restrict__ jp,
                                                            int64_t n) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const double h2 = *hn;
  const double s = h2 > 0.0 ? 1.0 / sqrt(h2) : 1.0;
  V[(int64_t)(*jp + 1) * n + k] = w[k] * s;
}

__global__ void k_set_j(int* jp, int v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *jp = v < 0 ? *jp + 1 : v;
}

struct GmresWs {
  double* V;     // [m + 1][n]
  double* u;     // [n] weighted operand
  double* w;     // [n] new Arnoldi vector before its projections
  double* part;  // [m + 1][nb]
  double* hd;    // [2 (m + 1) + 1]: first projection, second projection, squared norm
  int* jd;       // step index of the replayed Arnoldi step
  void* aws;     // sbd_apply workspace
  size_t aws_bytes;
  int nb;
};

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// basis, u, w, partials, projections, step index, apply workspace, then the sorted copies of
// b, x, the weights and the diagonal
size_t ws_bytes(int64_t n, int m, size_t apply_ws, int nb) {
  return align256((size_t)(m + 1) * n * 8) + 2 * align256((size_t)n * 8) + align256((size_t)(m + 1) * nb * 8) +
         align256((size_t)(2 * (m + 1) + 1) * 8) + 256 + align256(apply_ws) + 4 * align256((size_t)n * 8);
}

int num_partial_blocks(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>(1024, ceil_div(n, 4 * kThreads))); }

}  // namespace
}  // namespace sbd

using namespace sbd;

namespace {

struct Ctx {
  sbd_plan_t plan;
  int64_t n;
  const double* wts;
  const double* diag;
  GmresWs ws;
  hipStream_t st;
};

unsigned nblk(int64_t n) { return (unsigned)ceil_div(n, kThreads); }

// y = A v  (y must not alias v)
sbd_status op_apply(Ctx& c, const double* v, double* y) {
  hipLaunchKernelGGL(k_weight, dim3(nblk(c.n)), dim3(kThreads), 0, c.st, c.ws.u, c.wts, v, c.n);
  sbd_status s = sbd_apply_parts(c.plan, c.ws.u, y, 1, SBD_F64, SBD_PART_ALL | SBD_IO_SORTED, c.ws.aws,
                                  c.ws.aws_bytes, c.st);
  if (s != SBD_OK) return s;
  if (c.diag)
    hipLaunchKernelGGL(k_finish_op, dim3(nblk(c.n)), dim3(kThreads), 0, c.st, y, c.diag, v, 1.0,
                       (const double*)nullptr, c.n);
  return hipGetLastError() == hipSuccess ? SBD_OK : SBD_EHIP;
}

// out[0..cnt) = V[0..cnt) . w   (device)
void dots(Ctx& c, const double* V, int cnt, const double* w, double* out) {
  hipLaunchKernelGGL(k_dot_partials, dim3(c.ws.nb, cnt), dim3(kThreads), 0, c.st, V, c.n, w, c.n, c.ws.part);
  hipLaunchKernelGGL(k_reduce_partials, dim3(cnt), dim3(kThreads), 0, c.st, c.ws.part, c.ws.nb, out);
}

// One Arnoldi step with the step index read from c.ws.jd (recorded into a graph, or run
// directly): V[j + 1] = normalised projection of A V[j] against V[0..j].
sbd_status arnoldi_step(Ctx& c, int m) {
  const unsigned g = nblk(c.n);
  hipLaunchKernelGGL(k_weight_j, dim3(g), dim3(kThreads), 0, c.st, c.ws.u, c.wts, (const double*)c.ws.V,
                     (const int*)c.ws.jd, c.n);
  sbd_status s = sbd_apply_parts(c.plan, c.ws.u, c.ws.w, 1, SBD_F64, SBD_PART_ALL | SBD_IO_SORTED, c.ws.aws,
                                  c.ws.aws_bytes, c.st);
  if (s != SBD_OK) return s;
  if (c.diag)
    hipLaunchKernelGGL(k_diag_j, dim3(g), dim3(kThreads), 0, c.st, c.ws.w, c.diag, (const double*)c.ws.V,
                       (const int*)c.ws.jd, c.n);
  double* h1 = c.ws.hd;
  double* h2 = c.ws.hd + (m + 1);
  double* hn = c.ws.hd + 2 * (m + 1);
  for (double* h : {h1, h2}) {
    hipLaunchKernelGGL(k_dot_partials_j, dim3(c.ws.nb, m + 1), dim3(kThreads), 0, c.st, (const double*)c.ws.V, c.n,
                       (const double*)c.ws.w, c.n, (const int*)c.ws.jd, c.ws.part);
    hipLaunchKernelGGL(k_reduce_partials_j, dim3(m + 1), dim3(kThreads), 0, c.st, (const double*)c.ws.part, c.ws.nb,
                       (const int*)c.ws.jd, h);
    hipLaunchKernelGGL(k_gemv_j, dim3(g), dim3(kThreads), 0, c.st, c.ws.w, (const double*)c.ws.V, c.n,
                       (const double*)h, (const int*)c.ws.jd);
  }
  dots(c, c.ws.w, 1, c.ws.w, hn);
  hipLaunchKernelGGL(k_store_next_j, dim3(g), dim3(kThreads), 0, c.st, c.ws.V, (const double*)c.ws.w,
                     (const double*)hn, (const int*)c.ws.jd, c.n);
  hipLaunchKernelGGL(k_set_j, dim3(1), dim3(64), 0, c.st, c.ws.jd, -1);
  return hipGetLastError() == hipSuccess ? SBD_OK : SBD_EHIP;
}

// The step as a graph (nullptr if capture is not possible on this stream, e.g. the
// caller is capturing it already; the steps then run directly).
hipGraphExec_t capture_step(Ctx& c, int m) {
  if (plan_timing(c.plan)) return nullptr;  // per-launch timing events follow eager launches
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(c.st, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return nullptr;
  if (hipStreamBeginCapture(c.st, hipStreamCaptureModeThreadLocal) != hipSuccess) return nullptr;
  const sbd_status s = arnoldi_step(c, m);
  hipGraph_t graph = nullptr;
  const hipError_t e = hipStreamEndCapture(c.st, &graph);
  if (s != SBD_OK || e != hipSuccess || !graph) {
    if (graph) (void)hipGraphDestroy(graph);
    (void)hipGetLastError();
    return nullptr;
  }
  hipGraphExec_t exec = nullptr;
  if (hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) exec = nullptr;
  (void)hipGraphDestroy(graph);
  return exec;
}

sbd_status fetch(Ctx& c, double* host, const double* dev, int cnt) {
  if (hipMemcpyAsync(host, dev, cnt * sizeof(double), hipMemcpyDeviceToHost, c.st) != hipSuccess ||
      hipStreamSynchronize(c.st) != hipSuccess)
    return SBD_EHIP;
  return SBD_OK;
}

}  // namespace

extern "C" {

size_t sbd_gmres_workspace_bytes(sbd_plan_t plan, int restart) {
  if (!plan) return 0;
  int m = restart > 0 ? restart : 30;
  if (m > kMaxRestart) return 0;
  sbd_info info;
  if (sbd_plan_info(plan, &info) != SBD_OK) return 0;
  return ws_bytes(info.n, m, sbd_workspace_bytes(plan, 1), num_partial_blocks(info.n));
}

sbd_status sbd_gmres(sbd_plan_t plan, const double* weights, const double* diag, const double* b, double* x,
                     const sbd_gmres_options* opt_in, void* workspace, size_t workspace_bytes, void* stream,
                     int* iterations, double* relres) {
  if (iterations) *iterations = 0;
  if (relres) *relres = NAN;
  if (!plan || !b || !x) return fail_with(SBD_EINVAL, "NULL plan, b or x");
  sbd_info info;
  sbd_status s = sbd_plan_info(plan, &info);
  if (s != SBD_OK) return s;
  if (info.kind == SBD_HELMHOLTZ)
    return fail_with(SBD_EUNSUPPORTED, "sbd_gmres supports real kernels only (Laplace, general)");
  if (info.bipartite) return fail_with(SBD_EUNSUPPORTED, "sbd_gmres needs a square operator (a plan from sbd_plan)");
  sbd_gmres_options opt{30, 100, 1e-6, 0};
  if (opt_in) opt = *opt_in;
  const int m = opt.restart > 0 ? opt.restart : 30;
  const int cycles = opt.max_restarts > 0 ? opt.max_restarts : 100;
  const double rtol = opt.rtol > 0 ? opt.rtol : 1e-6;
  if (m > kMaxRestart) return fail_with(SBD_EINVAL, "restart above 64");
  Ctx c;
  c.plan = plan;
  c.n = info.n;
  c.wts = weights;
  c.diag = diag;
  c.st = (hipStream_t)stream;
  // a graph cannot be captured on the legacy default stream: the solve then runs on a
  // stream of its own that first waits for the caller's queued work
  hipStream_t own_stream = nullptr;
  if (!c.st) {
    hipEvent_t ev = nullptr;
    if (hipStreamCreateWithFlags(&own_stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess || hipEventRecord(ev, nullptr) != hipSuccess ||
        hipStreamWaitEvent(own_stream, ev, 0) != hipSuccess) {
      if (ev) (void)hipEventDestroy(ev);
      if (own_stream) (void)hipStreamDestroy(own_stream);
      return fail_with(SBD_EHIP, "GMRES stream");
    }
    (void)hipEventDestroy(ev);
    c.st = own_stream;
  }
  const int nb = num_partial_blocks(c.n);
  const size_t aws = sbd_workspace_bytes(plan, 1);
  const size_t need = ws_bytes(c.n, m, aws, nb);
  void* own = nullptr;
  AllocStream alloc_scope(c.st);  // the solve's own workspace is stream-ordered on its stream
  auto drop_stream = [&] {
    if (own_stream) {
      (void)hipStreamSynchronize(own_stream);
      (void)hipStreamDestroy(own_stream);
      own_stream = nullptr;
    }
  };
  if (workspace) {
    if (workspace_bytes < need) {
      drop_stream();
      return fail_with(SBD_EINVAL, "workspace too small");
    }
  } else {
    if (dev_malloc(&own, need) != hipSuccess) {
      drop_stream();
      return fail_with(SBD_ENOMEM, "GMRES workspace");
    }
    workspace = own;
  }
  auto* p = static_cast<unsigned char*>(workspace);
  c.ws.V = reinterpret_cast<double*>(p);
  p += align256((size_t)(m + 1) * c.n * 8);
  c.ws.u = reinterpret_cast<double*>(p);
  p += align256((size_t)c.n * 8);
  c.ws.w = reinterpret_cast<double*>(p);
  p += align256((size_t)c.n * 8);
  c.ws.part = reinterpret_cast<double*>(p);
  p += align256((size_t)(m + 1) * nb * 8);
  c.ws.hd = reinterpret_cast<double*>(p);
  p += align256((size_t)(2 * (m + 1) + 1) * 8);
  c.ws.jd = reinterpret_cast<int*>(p);
  p += 256;
  c.ws.aws = p;
  c.ws.aws_bytes = aws;
  c.ws.nb = nb;
  p += align256(aws);
  // sorted copies: b, x, weights, diagonal
  const int32_t* perm = plan_perm(plan);
  double* bs = reinterpret_cast<double*>(p);
  p += align256((size_t)c.n * 8);
  double* xs = reinterpret_cast<double*>(p);
  p += align256((size_t)c.n * 8);
  double* wsrt = reinterpret_cast<double*>(p);
  p += align256((size_t)c.n * 8);
  double* dsrt = reinterpret_cast<double*>(p);
  const unsigned gp = nblk(c.n);
  hipLaunchKernelGGL(k_gather_perm, dim3(gp), dim3(kThreads), 0, c.st, bs, b, perm, c.n);
  if (!opt.zero_guess) hipLaunchKernelGGL(k_gather_perm, dim3(gp), dim3(kThreads), 0, c.st, xs, (const double*)x, perm, c.n);
  if (weights) hipLaunchKernelGGL(k_gather_perm, dim3(gp), dim3(kThreads), 0, c.st, wsrt, weights, perm, c.n);
  if (diag) hipLaunchKernelGGL(k_gather_perm, dim3(gp), dim3(kThreads), 0, c.st, dsrt, diag, perm, c.n);
  c.wts = weights ? wsrt : nullptr;
  c.diag = diag ? dsrt : nullptr;
  double* const x_user = x;
  b = bs;
  x = xs;
  hipGraphExec_t step_graph = nullptr;
  auto done = [&](sbd_status r) {
    hipLaunchKernelGGL(k_scatter_perm, dim3(gp), dim3(kThreads), 0, c.st, x_user, (const double*)xs, perm, c.n);
    (void)hipStreamSynchronize(c.st);
    if (step_graph) (void)hipGraphExecDestroy(step_graph);
    if (own) dev_free(own);
    (void)hipStreamSynchronize(c.st);
    drop_stream();
    return r;
  };
  const unsigned g = nblk(c.n);
  double* V = c.ws.V;
  std::vector<double> hh(2 * (m + 1) + 1), H((size_t)(m + 1) * m), cs(m), sn(m), gv(m + 1), y(m);
  // ||b||
  dots(c, b, 1, b, c.ws.hd);
  double bn2;
  if ((s = fetch(c, &bn2, c.ws.hd, 1)) != SBD_OK) return done(fail_with(s, "GMRES norm"));
  const double bnorm = std::sqrt(bn2);
  if (opt.zero_guess) (void)hipMemsetAsync(x, 0, (size_t)c.n * 8, c.st);
  if (bnorm == 0.0) {
    (void)hipMemsetAsync(x, 0, (size_t)c.n * 8, c.st);
    if (relres) *relres = 0.0;
    return done(SBD_OK);
  }
  int total = 0;
  double res = NAN;
  bool have_res = false;
  bool graph_tried = false;
  for (int cyc = 0; cyc < cycles; ++cyc) {
    // r = b - A x  into V[0]
    if (opt.zero_guess && cyc == 0) {
      (void)hipMemcpyAsync(V, b, (size_t)c.n * 8, hipMemcpyDeviceToDevice, c.st);
    } else {
      if ((s = op_apply(c, x, V)) != SBD_OK) return done(s);
      hipLaunchKernelGGL(k_finish_op, dim3(g), dim3(kThreads), 0, c.st, V, (const double*)nullptr, (const double*)x,
                         -1.0, b, c.n);
    }
    dots(c, V, 1, V, c.ws.hd);
    double r2;
    if ((s = fetch(c, &r2, c.ws.hd, 1)) != SBD_OK) return done(fail_with(s, "GMRES residual"));
    const double beta = std::sqrt(r2);
    res = beta / bnorm;
    have_res = true;
    if (res <= rtol) break;
    have_res = false;
    hipLaunchKernelGGL(k_scale, dim3(g), dim3(kThreads), 0, c.st, V, V, 1.0 / beta, c.n);
    std::fill(gv.begin(), gv.end(), 0.0);
    gv[0] = beta;
    int k = 0;
    bool conv = false;
    hipLaunchKernelGGL(k_set_j, dim3(1), dim3(64), 0, c.st, c.ws.jd, 0);
    if (!step_graph && !graph_tried) {
      graph_tried = true;
      step_graph = capture_step(c, m);
    }
    for (int j = 0; j < m; ++j) {
      if (step_graph) {
        if (hipGraphLaunch(step_graph, c.st) != hipSuccess) return done(fail_with(SBD_EHIP, "GMRES step graph"));
      } else if ((s = arnoldi_step(c, m)) != SBD_OK) {
        return done(s);
      }
      if ((s = fetch(c, hh.data(), c.ws.hd, 2 * (m + 1) + 1)) != SBD_OK) return done(fail_with(s, "GMRES step"));
      double* col = &H[(size_t)j * (m + 1)];
      for (int i = 0; i <= j; ++i) col[i] = hh[i] + hh[(m + 1) + i];
      const double hnext = std::sqrt(std::max(0.0, hh[2 * (m + 1)]));
      col[j + 1] = hnext;
      for (int i = 0; i < j; ++i) {  // earlier rotations
        double t = cs[i] * col[i] + sn[i] * col[i + 1];
        col[i + 1] = -sn[i] * col[i] + cs[i] * col[i + 1];
        col[i] = t;
      }
      double den = std::hypot(col[j], col[j + 1]);
      cs[j] = den > 0 ? col[j] / den : 1.0;
      sn[j] = den > 0 ? col[j + 1] / den : 0.0;
      col[j] = den;
      col[j + 1] = 0.0;
      gv[j + 1] = -sn[j] * gv[j];
      gv[j] = cs[j] * gv[j];
      ++total;
      k = j + 1;
      if (std::fabs(gv[j + 1]) <= rtol * bnorm || hnext == 0.0) {
        conv = true;
        break;
      }
    }
    // y = H(0:k, 0:k)^-1 g, x += V(:, 0:k) y
    for (int i = k - 1; i >= 0; --i) {
      double t = gv[i];
      for (int l = i + 1; l < k; ++l) t -= H[(size_t)l * (m + 1) + i] * y[l];
      y[i] = t / H[(size_t)i * (m + 1) + i];
    }
    if (hipMemcpyAsync(c.ws.hd, y.data(), k * sizeof(double), hipMemcpyHostToDevice, c.st) != hipSuccess)
      return done(fail_with(SBD_EHIP, "GMRES update"));
    hipLaunchKernelGGL(k_gemv_acc, dim3(g), dim3(kThreads), 0, c.st, x, (const double*)V, c.n, c.n,
                       (const double*)c.ws.hd, k, 1.0);
    if (hipStreamSynchronize(c.st) != hipSuccess) return done(fail_with(SBD_EHIP, "GMRES update"));
    (void)conv;
  }
  if (!have_res) {  // cycles exhausted: true residual of the returned x
    if ((s = op_apply(c, x, V)) != SBD_OK) return done(s);
    hipLaunchKernelGGL(k_finish_op, dim3(g), dim3(kThreads), 0, c.st, V, (const double*)nullptr, (const double*)x,
                       -1.0, b, c.n);
    dots(c, V, 1, V, c.ws.hd);
    double r2;
    if ((s = fetch(c, &r2, c.ws.hd, 1)) != SBD_OK) return done(fail_with(s, "GMRES residual"));
    res = std::sqrt(r2) / bnorm;
  }
  if (iterations) *iterations = total;
  if (relres) *relres = res;
  if (hipGetLastError() != hipSuccess) return done(fail_with(SBD_EHIP, "GMRES kernels"));
  return done(res <= rtol ? SBD_OK : fail_with(SBD_ENOCONV, "GMRES stopped above rtol"));
}

}  // extern "C"
