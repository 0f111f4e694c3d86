// C ABI of the SBD matvec: plan (off-line part) and apply (on-line part) of
// Section 1 of the paper, orchestrating the host FP64 fit and the HIP kernels.
//
// Far field.  With phi the exponential-of-semicircle spreading kernel on an
// x-grid of spacing h, every plane wave satisfies
//   exp(i z.xi) ~ h^2 / phi_hat(xi) * sum_g phi(x_g - z) exp(i x_g.xi),  |xi| <= S,
// so NUFFT_+(omega_hat * NUFFT_-(f)) (eq. "far convolution") becomes
//   q_far(z_k) = sum_g phi(x_g - z_k) [H * F](x_g),  F = sum_l f_l phi(x_g - z_l),
//   H(x_g) = h^4 sum_nu omega_hat_nu exp(i x_g.xi_nu) / phi_hat(xi_nu)^2,
// a linear convolution on the grid (Toeplitz in both axes).  The plan builds
// H from the concentric-circle frequencies xi_nu of Section 5 (a type-1 NUFFT
// at plan time) and stores its zero-padded DFT; the apply is spread ->
// FFT -> multiply -> inverse FFT -> interpolate, plus the close correction.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstring>
#include <map>
#include <mutex>
#include <set>
#include <tuple>
#include <string>
#include <thread>
#include <vector>

#include "../../include/sbd.h"
#include "colconv.h"
#include "common.h"
#include "rows.h"
#include "fft.h"
#include "host/layout.h"
#include "host/sbd_fit.h"
#include "kernels.h"

namespace sbd {

static thread_local std::string g_last_error;

void set_last_error(const char* what, const char* file, int line) {
  g_last_error = std::string(what) + " (" + file + ":" + std::to_string(line) + ")";
}

struct LaunchMark {
  std::string name;
  hipEvent_t ev;
  double bytes;
};
struct LaunchMarks {
  std::vector<LaunchMark> marks;
};
static thread_local LaunchMarks* g_marks = nullptr;

void mark_launch(const char* name, hipStream_t st, double bytes) {
  if (!g_marks) return;
  hipEvent_t e;
  if (hipEventCreate(&e) != hipSuccess) return;
  (void)hipEventRecord(e, st);
  g_marks->marks.push_back(LaunchMark{name, e, bytes});
}

static thread_local hipStream_t g_alloc_st = nullptr;
static thread_local bool g_alloc_set = false;

AllocStream::AllocStream(hipStream_t st) : prev(g_alloc_st), prev_set(g_alloc_set) {
  g_alloc_st = st;
  g_alloc_set = true;
}
AllocStream::~AllocStream() {
  g_alloc_st = prev;
  g_alloc_set = prev_set;
}

// ---- large-block cache (sbd_set_cache_limit)
// While the limit is positive: blocks of at least kCacheMin bytes come from the stream-ordered
// allocator in size classes 2^(k/4) (rounded to 2 MiB) and, released, wait in a per-device
// free list for a later request of the same class, up to g_cache_limit bytes in all (the
// largest classes are evicted first).  Only idle blocks enter the list: one released inside an
// AllocStream scope waits for its stream first (plan temporaries are released after their
// kernels have been waited for anyway), one released outside a scope is idle by contract
// (sbd_free of an idle plan), so a block taken from the list needs no ordering.  Every release
// in this mode is stream-ordered (hipFreeAsync, on the legacy stream outside a scope): no
// release waits for the whole device, which would break a graph another thread captures.
namespace {
constexpr size_t kCacheMin = (size_t)32 << 20;
struct CachedBlock {
  void* p;
  int dev;
};
std::mutex g_cache_mu;
size_t g_cache_limit = 0, g_cache_held = 0;
std::multimap<size_t, CachedBlock> g_cache;   // class bytes -> idle block
std::map<void*, size_t> g_cache_live;         // cache-class blocks in use -> class bytes
std::set<void*> g_pool_blocks;                // other blocks from the stream-ordered allocator

size_t cache_class(size_t bytes) {
  const double k = std::ceil(4.0 * std::log2((double)bytes));
  size_t c = (size_t)std::ceil(std::exp2(k / 4.0));
  const size_t g = (size_t)2 << 20;
  c = (c + g - 1) / g * g;
  return std::max(c, bytes);
}

// releases cached blocks (largest first) until at most `keep` bytes remain; caller holds the lock
void cache_trim(size_t keep) {
  while (g_cache_held > keep && !g_cache.empty()) {
    auto it = std::prev(g_cache.end());
    int cur = 0;
    (void)hipGetDevice(&cur);
    if (cur != it->second.dev) (void)hipSetDevice(it->second.dev);
    (void)hipFreeAsync(it->second.p, nullptr);
    if (cur != it->second.dev) (void)hipSetDevice(cur);
    g_cache_held -= it->first;
    g_cache.erase(it);
  }
}
}  // namespace

hipError_t dev_malloc(void** p, size_t bytes) {
  if (bytes == 0) bytes = 16;
  hipStream_t st = g_alloc_set ? g_alloc_st : nullptr;
  bool cache_on, pooled = g_alloc_set;
  size_t cls = 0;
  {
    std::lock_guard<std::mutex> g(g_cache_mu);
    cache_on = g_cache_limit > 0;
    if (cache_on && bytes >= kCacheMin) {
      int dev = 0;
      (void)hipGetDevice(&dev);
      cls = cache_class(bytes);
      auto range = g_cache.equal_range(cls);
      for (auto it = range.first; it != range.second; ++it) {
        if (it->second.dev != dev) continue;
        *p = it->second.p;
        g_cache.erase(it);
        g_cache_held -= cls;
        g_cache_live[*p] = cls;
        return hipSuccess;
      }
    }
  }
  if (cache_on) pooled = true;
  if (!pooled) return hipMalloc(p, bytes);
  hipError_t e = hipMallocAsync(p, cls ? cls : bytes, st);
  if (e == hipSuccess) {
    std::lock_guard<std::mutex> g(g_cache_mu);
    if (cls) g_cache_live[*p] = cls;
    else g_pool_blocks.insert(*p);
  }
  return e;
}

void dev_free(void* p) {
  if (!p) return;
  hipStream_t st = g_alloc_set ? g_alloc_st : nullptr;
  size_t cls = 0;
  bool pooled = false, cache_on = false;
  {
    std::lock_guard<std::mutex> g(g_cache_mu);
    cache_on = g_cache_limit > 0;
    auto it = g_cache_live.find(p);
    if (it != g_cache_live.end()) {
      cls = it->second;
      g_cache_live.erase(it);
    } else {
      auto pb = g_pool_blocks.find(p);
      if (pb != g_pool_blocks.end()) {
        g_pool_blocks.erase(pb);
        pooled = true;
      }
    }
  }
  if (cls && cache_on) {
    if (g_alloc_set) (void)hipStreamSynchronize(st);  // only idle blocks are cached
    int dev = 0;
    (void)hipGetDevice(&dev);
    std::lock_guard<std::mutex> g(g_cache_mu);
    g_cache.emplace(cls, CachedBlock{p, dev});
    g_cache_held += cls;
    cache_trim(g_cache_limit);
    return;
  }
  if (cls || pooled) {
    // outside a scope with the cache off, keep the device-wide wait of hipFree (the plan's
    // queued work may still use the block)
    if (g_alloc_set || cache_on) (void)hipFreeAsync(p, st);
    else (void)hipFree(p);
    return;
  }
  (void)hipFree(p);
}

hipError_t dev_upload(void* dst, const void* src, size_t bytes) {
  // blocking, ordered on the allocation stream (after the stream-ordered allocation)
  return g_alloc_set ? hipMemcpyWithStream(dst, src, bytes, hipMemcpyHostToDevice, g_alloc_st)
                     : hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice);
}

sbd_status fail_with(sbd_status st, const char* msg) {
  g_last_error = msg;
  return st;
}

static sbd_status fail(sbd_status st, const std::string& msg) {
  g_last_error = msg;
  return st;
}

namespace {

constexpr double kPi = 3.14159265358979323846;
size_t g_max_lds = 0;
size_t max_lds() {
  if (g_max_lds) return g_max_lds;
  int dev = 0, v = 0;
  if (hipGetDevice(&dev) == hipSuccess &&
      hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && v > 0)
    g_max_lds = std::min<size_t>((size_t)v, 160 * 1024);
  else
    g_max_lds = 65536;
  return g_max_lds;
}

// Process-wide cache of SBD fits for plans made with fit_reuse.  A fit of the
// unit-scaled shape on [a', 1] with a' <= a meets the same bound on [a, 1], so
// a is rounded down to the grid 2^(-k/8) and fits are shared by key.
using FitKey = std::tuple<int, double, double, double, int>;  // kind, eps, a', kappa, forced P
std::mutex g_fit_mu;
std::map<FitKey, FitResult> g_fit_cache;

int cached_fit(int kind, double a, double eps, double kappa, int force_P, int nthreads, bool reuse,
               FitResult& out, std::string& msg) {
  if (!reuse) return sbd_fit(kind, a, eps, kappa, force_P, nthreads, out, msg);
  const double ar = std::exp2(std::floor(std::log2(a) * 8.0) / 8.0);
  FitKey key{kind, eps, ar, kappa, force_P};
  {
    std::lock_guard<std::mutex> g(g_fit_mu);
    auto it = g_fit_cache.find(key);
    if (it != g_fit_cache.end()) {
      out = it->second;
      return 0;
    }
  }
  int rc = sbd_fit(kind, ar, eps, kappa, force_P, nthreads, out, msg);
  if (rc == 0) {
    std::lock_guard<std::mutex> g(g_fit_mu);
    g_fit_cache.emplace(key, out);
  }
  return rc;
}

// Worst-case 1-D plane-wave reconstruction error of spreading + deconvolution
// with the ES kernel, tabulated by kernel width w = 3..16 for three x-grid
// oversampling factors (measured over |xi| <= S and all sub-cell positions,
// shape parameter beta = ratio * w).
struct EsTable {
  double sigma;
  double ratio;
  double err[14];
};
const EsTable kEsTables[3] = {
    {1.25, 1.80, {8.7e-2, 1.6e-2, 6.2e-3, 1.7e-3, 4.9e-4, 1.8e-4, 4.2e-5, 8.7e-6, 2.7e-6, 6.8e-7, 2.5e-7, 8.2e-8, 2.2e-8, 5.3e-9}},
    {1.50, 2.02, {3.3e-2, 5.5e-3, 1.1e-3, 2.1e-4, 4.6e-5, 5.8e-6, 1.3e-6, 2.7e-7, 4.4e-8, 9.2e-9, 2.0e-9, 2.9e-10, 3.6e-11, 6.4e-12}},
    {2.00, 2.25, {9.4e-3, 1.5e-3, 1.7e-4, 2.6e-5, 2.7e-6, 3.8e-7, 4.5e-8, 5.1e-9, 7.8e-10, 7.7e-11, 7.4e-12, 9.4e-13, 1.3e-13, 2.2e-14}},
};

void es_params(double sigma_req, double tol, double* sigma, int* w, double* beta) {
  int t = 0;
  double best = 1e9;
  for (int i = 0; i < 3; ++i)
    if (std::fabs(kEsTables[i].sigma - sigma_req) < best) { best = std::fabs(kEsTables[i].sigma - sigma_req); t = i; }
  const EsTable& T = kEsTables[t];
  int wsel = 16;
  for (int k = 0; k < 14; ++k)
    if (T.err[k] <= tol) { wsel = k + 3; break; }
  *sigma = T.sigma;
  *w = wsel;
  *beta = T.ratio * wsel;
}

template <typename F>
void host_parallel_for(int64_t n, F&& f) {
  int nt = (int)std::min<unsigned>(16, std::max(1u, std::thread::hardware_concurrency()));
  std::vector<std::thread> th;
  int64_t chunk = (n + nt - 1) / nt;
  for (int t = 0; t < nt; ++t) {
    int64_t s = t * chunk, e = std::min(n, s + chunk);
    if (s >= e) break;
    th.emplace_back([=, &f] { for (int64_t i = s; i < e; ++i) f(i); });
  }
  for (auto& x : th) x.join();
}

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

}  // namespace

struct Plan {
  int device = 0;              // the HIP device current when the plan was made (its memory's)
  int64_t n = 0;
  int kind = 0;                // kernel of the apply path: a general kernel runs as a real (Laplace-like) one
  bool general = false;        // SBD_GENERAL: own fit, far weights and near tables
  GeneralKernel gk;
  double wavenumber = 0;
  int precision = 0;
  int max_rhs = 1;
  double eps = 0;
  double delta_min = 0, delta_max = 0, cx = 0, cy = 0;
  FitResult fit;
  Layout L;
  double sigma = 1.25;
  double d2max = 0;
  int64_t n_xi = 0, nnz = 0;
  size_t byte_cap = 0;
  double nufft_tol = 0;        // spreading-kernel tolerance of the apply
  // device arrays
  int32_t* perm = nullptr;
  int32_t* tile_start = nullptr;
  // targets (aliases of perm / skeys / loc for a single point set)
  int64_t n_tgt = 0;
  int bipartite = 0;
  int32_t* tperm = nullptr;
  int32_t* tskeys = nullptr;
  void* tloc = nullptr;
  int32_t* unit_tile = nullptr;   // interpolation work units (see kUnitPoints)
  int32_t* unit_start = nullptr;
  int64_t nunits = 0;
  void* loc = nullptr;
  int64_t* row_ptr = nullptr;
  int32_t* col = nullptr;
  double* val = nullptr;       // FP64 D (every plan except FP32 ones made with near_fp32)
  float* valf = nullptr;       // D rounded to FP32 (near_fp32 plans; replaces val)
  int near_fp32 = 0;
  int deterministic = 0;
  int near_assembly = 0;       // 1: D by the pair-difference NUFFT
  double pd_tol = 0;           // its tolerance
  int pd_grid = 0;             // its frequency-grid edge
  double near_seconds = 0, assembly_seconds = 0, bin_seconds = 0, symbol_seconds = 0;
  int32_t* skeys = nullptr;
  void* symbol = nullptr;      // [My][Mx] real T or complex T, apply storage order
  int symbol_complex = 0;
  double self_im = 0;
  AxisPlan apx, apy;
  ColConvPlan cc;             // compiled whole-column convolution for My (symbol in column layout)
  RowPlan rr;                 // compiled real-row transforms for Mx (Laplace, real f)
  RealRowPlan rrp;
  int real_rows = 0;          // real-data row transforms available (Laplace, real f)
  int row_pairs = 1;          // compiled transforms may interleave the row spectra in pairs
                              // (SBD_ROW_PAIRS=0 at plan time keeps natural rows)
  // per-launch timing (sbd_options.timing)
  int timing = 0;
  LaunchMarks marks;
  std::vector<std::string> t_names;
  std::vector<double> t_ms;
  std::vector<double> t_bytes;
  std::vector<int64_t> t_cnt;
  int64_t t_calls = 0;
  // internal workspace
  void* ws = nullptr;
  size_t ws_bytes = 0;
  double plan_seconds = 0, fit_seconds = 0;
  size_t resident = 0;
  std::vector<void*> owned;

  std::mutex owned_mu;          // alloc / release run on the plan's two building threads
  hipError_t alloc(void** p, size_t bytes) {
    hipError_t e = dev_malloc(p, bytes);
    if (e == hipSuccess) {
      std::lock_guard<std::mutex> g(owned_mu);
      owned.push_back(*p);
      resident += bytes;
    }
    return e;
  }
  // free one allocation made by alloc before the plan ends
  void release(void* p, size_t bytes) {
    std::lock_guard<std::mutex> g(owned_mu);
    auto it = std::find(owned.begin(), owned.end(), p);
    if (it == owned.end()) return;
    owned.erase(it);
    resident -= bytes;
    dev_free(p);
  }
  void drain_marks() {
    if (marks.marks.empty()) return;
    (void)hipEventSynchronize(marks.marks.back().ev);
    for (size_t i = 1; i < marks.marks.size(); ++i) {
      const std::string& nm = marks.marks[i].name;
      if (nm == "begin") continue;
      float ms = 0;
      (void)hipEventElapsedTime(&ms, marks.marks[i - 1].ev, marks.marks[i].ev);
      size_t k = 0;
      while (k < t_names.size() && t_names[k] != nm) ++k;
      if (k == t_names.size()) { t_names.push_back(nm); t_ms.push_back(0); t_bytes.push_back(0); t_cnt.push_back(0); }
      t_ms[k] += ms;
      t_bytes[k] += marks.marks[i].bytes;
      t_cnt[k] += 1;
    }
    for (auto& m : marks.marks) (void)hipEventDestroy(m.ev);
    marks.marks.clear();
  }
  ~Plan() {
    // the plan's device is current while its memory is released (a cached block is filed
    // under the current device)
    int cur = -1;
    if (hipGetDevice(&cur) == hipSuccess && cur != device) (void)hipSetDevice(device);
    else cur = -1;
    release_all();
    if (cur >= 0) (void)hipSetDevice(cur);
  }
  void release_all() {
    drain_marks();
    // with the cache on, the plan is idle by contract (sbd_free): its blocks are reused or
    // released stream-ordered, with no device-wide wait
    for (void* p : owned) dev_free(p);
    if (ws) dev_free(ws);
    free_axis_plan(apx);
    free_axis_plan(apy);
    free_colconv_plan(cc);
    free_row_plan(rr);
    free_real_row_plan(rrp);
  }
};

bool plan_timing(sbd_plan_t plan) { return plan && reinterpret_cast<Plan*>(plan)->timing != 0; }

const int32_t* plan_perm(sbd_plan_t plan) { return plan ? reinterpret_cast<Plan*>(plan)->perm : nullptr; }

namespace {

size_t elem_real(int precision) { return precision ? 8 : 4; }

struct WsLayout {
  size_t sub = 0, grid = 0, fs = 0, qn = 0, total = 0;
};

WsLayout ws_layout(const Plan& p, int nrhs) {
  WsLayout w;
  size_t er = elem_real(p.precision);
  size_t ntiles = (size_t)p.L.ntx * p.L.nty;
  int cp = (p.kind == 1) ? 2 : 2;  // complex capacity (complex f is allowed for both kernels)
  auto al = [](size_t b) { return (b + 255) / 256 * 256; };
  w.sub = al(ntiles * (size_t)p.L.SG * p.L.SG * er * cp * nrhs);
  w.grid = al((size_t)p.L.Mx * p.L.My * er * 2 * nrhs);
  w.fs = al((size_t)p.n * er * cp * nrhs);
  // close-correction sums of several right-hand sides (k_near_multi)
  w.qn = nrhs > 1 ? al((size_t)p.n_tgt * 8 * cp * nrhs) : 0;
  w.total = w.sub + w.grid + w.fs + w.qn;
  return w;
}

// The sparse spectrum (Section 1, eq. "Gapprox"): circles of radius rho_p / delta_max with
// M_p nodes of weight alpha_p / M_p each (times the kernel's constant), plus the xi = 0 node
// of the Laplace constant term or the circle |xi| = k carrying (i/4) J0(k r) for Helmholtz.
void far_spectrum(const Plan& P, std::vector<double>& radius, std::vector<int64_t>& Mc, std::vector<double2>& wgt) {
  const FitResult& F = P.fit;
  const double cg = P.general ? 1.0 : P.kind == 0 ? -1.0 / (2.0 * kPi) : -0.25;
  for (int p = 0; p < F.P; ++p) {
    radius.push_back(F.radii[p] / P.delta_max);
    Mc.push_back(F.M[p]);
    wgt.push_back(make_double2(cg * F.coef[p] / (double)F.M[p], 0.0));
  }
  if (P.kind == 0) {
    radius.push_back(0.0);
    Mc.push_back(1);
    wgt.push_back(make_double2(P.general ? F.constant : -std::log(P.delta_max) / (2.0 * kPi), 0.0));
  } else {
    radius.push_back(P.wavenumber);
    Mc.push_back(F.extra_M);
    wgt.push_back(make_double2(0.0, 0.25 / (double)F.extra_M));
  }
}

// Close-correction entries by the pair-difference NUFFT (Section 1, eq. "defD"; Section
// 6.1, eq. "Complex:assemble"): the value of every stored pair is recomputed as
// G(y) - sum_nu omega_hat_nu exp(i y . xi_nu) at y = target - source, the sum over every
// circle node taken as a type-3 NUFFT in FP64 at tolerance pd_tol.
sbd_status assemble_pairdiff(Plan& P, const double2* xt, const double2* xs, hipStream_t st) {
  if (P.general) return fail(SBD_EUNSUPPORTED, "near_assembly = 1 supports SBD_LAPLACE and SBD_HELMHOLTZ only");
  std::vector<double> radius;
  std::vector<int64_t> Mc;
  std::vector<double2> wgt;
  far_spectrum(P, radius, Mc, wgt);
  const int nc = (int)radius.size();
  std::vector<int64_t> start(nc + 1, 0);
  for (int c = 0; c < nc; ++c) start[c + 1] = start[c] + Mc[c];
  double S = 0;
  for (double r : radius) S = std::max(S, r);
  double sig, beta;
  int w;
  es_params(2.0, P.pd_tol, &sig, &w, &beta);
  PdArgs a;
  a.ncirc = nc;
  a.nnodes = start[nc];
  a.h = kPi / (2.0 * P.delta_min);  // |h y| <= pi / 2 on every stored pair
  a.w = w;
  a.beta = beta;
  a.J = (int)std::ceil(S / a.h + 0.5 * w);
  a.G = (int)(8 * ceil_div(2 * (int64_t)a.J + 2, 8));
  if (a.G > kPdMaxGrid)
    return fail(SBD_EUNSUPPORTED, "near_assembly = 1: frequency grid of " + std::to_string(a.G) +
                                      " cells per axis exceeds 48 (delta_min times the largest circle radius too large)");
  P.pd_grid = a.G;
  const double tmax = a.h * P.delta_min * (1.0 + 1e-9);
  const int deg = 48;
  std::vector<double> cheb = es_hat_cheb(beta, 0.5 * w, tmax, deg);
  const int64_t nparts = pd_partials(a.nnodes);
  void *d_rad = nullptr, *d_start = nullptr, *d_w = nullptr, *d_cheb = nullptr, *d_part = nullptr, *d_b = nullptr;
  auto freeall = [&] {
    for (void* q : {d_rad, d_start, d_w, d_cheb, d_part, d_b})
      if (q) dev_free(q);
  };
  const size_t cells = (size_t)a.G * a.G;
  if (dev_malloc(&d_rad, nc * 8) || dev_malloc(&d_start, (nc + 1) * 8) || dev_malloc(&d_w, nc * 16) ||
      dev_malloc(&d_cheb, (deg + 1) * 8) || dev_malloc(&d_part, (size_t)nparts * cells * 16) ||
      dev_malloc(&d_b, cells * 16)) {
    freeall();
    return fail(SBD_ENOMEM, "pair-difference assembly buffers");
  }
  if (dev_upload(d_rad, radius.data(), nc * 8) || dev_upload(d_start, start.data(), (nc + 1) * 8) ||
      dev_upload(d_w, wgt.data(), nc * 16) || dev_upload(d_cheb, cheb.data(), (deg + 1) * 8)) {
    freeall();
    return fail(SBD_EHIP, "pair-difference assembly upload");
  }
  a.radius = (const double*)d_rad;
  a.node_start = (const int64_t*)d_start;
  a.weight = (const double2*)d_w;
  int rc = launch_pd_spread(a, (double2*)d_part, st);
  if (!rc) rc = launch_pd_reduce((const double2*)d_part, nparts, a.G, (double2*)d_b, st);
  if (!rc)
    rc = launch_pd_eval(a, (const double2*)d_b, (const double*)d_cheb, deg, tmax, xt, xs, P.row_ptr, P.col, P.n_tgt,
                        P.nnz, P.bipartite ? 0 : 1, P.kind, P.wavenumber, P.val, st);
  hipError_t se = hipStreamSynchronize(st);
  freeall();
  if (rc || se != hipSuccess)
    return fail(SBD_EHIP, std::string("pair-difference assembly kernels failed: ") + hipGetErrorString(se));
  return SBD_OK;
}

template <typename T>
sbd_status build_symbol(Plan& P, hipStream_t st) {
  // Type-1 NUFFT at plan time: H(g) = sum_nu c_nu exp(i g . theta_nu), theta = h xi.  Every
  // circle has an even number of equispaced nodes, so its node set is symmetric under
  // xi_x -> -xi_x and xi_y -> -xi_y and H is even in g_x and in g_y: only the quadrant
  // 0 <= g < n is computed, as the modes g' = g - s, |g'| <= n / 2, s = n / 2, of the node
  // sum with weights c_nu exp(i s . theta_nu), from a fine grid of size K >= 2 n per axis
  // (a quarter of the fine grid the whole window |g| < n would need).
  const Layout& L = P.L;
  // the symbol carries 1e-3 of the apply's NUFFT tolerance (at most 1e-6), floored at
  // what the precision resolves
  const double tol_t = std::max(P.precision ? 1e-12 : 1e-9, std::min(1e-6, 1e-3 * P.nufft_tol));
  double sig_t, beta_t;
  int wt;
  es_params(2.0, tol_t, &sig_t, &wt, &beta_t);
  // nodes sit within |theta| <= h S = pi / sigma, i.e. K / (2 sigma) fine cells of the centre:
  // K (1 - 1 / sigma) >= wt + 2 keeps every footprint inside one period (no wrap-around)
  const int64_t Kmin = (int64_t)std::ceil((wt + 2) / (1.0 - 1.0 / P.sigma));
  const int64_t Kx = next_smooth(std::max(2 * L.nx, Kmin)), Ky = next_smooth(std::max(2 * L.ny, Kmin));
  const int64_t sx = L.nx / 2, sy = L.ny / 2;
  AxisPlan fx, fy, ex, ey;
  auto cleanup = [&] { free_axis_plan(fx); free_axis_plan(fy); free_axis_plan(ex); free_axis_plan(ey); };
  if (build_axis_plan(fx, Kx, true, max_lds(), 1) || build_axis_plan(fy, Ky, true, max_lds(), 16) ||
      build_axis_plan(ex, L.Mx, true, max_lds(), 1) || build_axis_plan(ey, L.My, true, max_lds(), 16)) {
    cleanup();
    return fail(SBD_ENOMEM, "FFT plan for the grid symbol failed");
  }
  std::vector<double> radius;
  std::vector<int64_t> Mc;
  std::vector<double2> wgt;
  far_spectrum(P, radius, Mc, wgt);
  int64_t nxi = 0;
  for (size_t c = 0; c < radius.size(); ++c) nxi += Mc[c];
  P.n_xi = nxi;
  {
    // the tiled spreading finds circles by radius: sort all three arrays by radius
    std::vector<size_t> ord(radius.size());
    for (size_t c = 0; c < ord.size(); ++c) ord[c] = c;
    std::stable_sort(ord.begin(), ord.end(), [&](size_t x, size_t y) { return radius[x] < radius[y]; });
    std::vector<double> r2(ord.size());
    std::vector<int64_t> m2(ord.size());
    std::vector<double2> w2(ord.size());
    for (size_t c = 0; c < ord.size(); ++c) { r2[c] = radius[ord[c]]; m2[c] = Mc[ord[c]]; w2[c] = wgt[ord[c]]; }
    radius.swap(r2);
    Mc.swap(m2);
    wgt.swap(w2);
  }
  double smax = 0;
  for (double r : radius) smax = std::max(smax, r);
  const double alpha = 0.5 * L.w * L.h;
  const int cdeg = 48;
  std::vector<double> cheb = es_hat_cheb(L.beta, alpha, smax * (1.0 + 1e-9), cdeg);
  // psi_hat on the fine grids: psi(t) = es(t / alpha_t), alpha_t = wt Delta / 2, Delta = 2 pi / K
  auto invpsi = [&](int64_t K, int64_t n) {
    std::vector<double> v(n);
    double D = 2.0 * kPi / (double)K;
    double at = 0.5 * wt * D;
    host_parallel_for(n, [&](int64_t g) { v[g] = D / es_hat(beta_t, at, (double)g); });
    return v;
  };
  std::vector<double> ipx = invpsi(Kx, L.nx), ipy = invpsi(Ky, L.ny);
  void *d_rad = nullptr, *d_M = nullptr, *d_w = nullptr, *d_cheb = nullptr,
       *d_ipx = nullptr, *d_ipy = nullptr, *d_fine = nullptr, *d_emb = nullptr;
  auto freeall = [&] {
    for (void* q : {d_rad, d_M, d_w, d_cheb, d_ipx, d_ipy, d_fine, d_emb})
      if (q) dev_free(q);
    cleanup();
  };
  size_t fine_bytes = (size_t)Kx * Ky * sizeof(double2);
  size_t emb_bytes = (size_t)L.Mx * L.My * sizeof(double2);
  if (dev_malloc(&d_rad, radius.size() * 8) ||
      dev_malloc(&d_M, Mc.size() * 8) || dev_malloc(&d_w, wgt.size() * 16) || dev_malloc(&d_cheb, cheb.size() * 8) ||
      dev_malloc(&d_ipx, ipx.size() * 8) || dev_malloc(&d_ipy, ipy.size() * 8) || dev_malloc(&d_fine, fine_bytes) ||
      dev_malloc(&d_emb, emb_bytes)) {
    freeall();
    return fail(SBD_ENOMEM, "device allocation for the grid symbol failed");
  }
  bool ok = dev_upload(d_rad, radius.data(), radius.size() * 8) == hipSuccess &&
            dev_upload(d_M, Mc.data(), Mc.size() * 8) == hipSuccess &&
            dev_upload(d_w, wgt.data(), wgt.size() * 16) == hipSuccess &&
            dev_upload(d_cheb, cheb.data(), cheb.size() * 8) == hipSuccess &&
            dev_upload(d_ipx, ipx.data(), ipx.size() * 8) == hipSuccess &&
            dev_upload(d_ipy, ipy.data(), ipy.size() * 8) == hipSuccess;
  if (!ok) {
    freeall();
    return fail(SBD_EHIP, "upload of symbol tables failed");
  }
  NodeSpreadArgs na;
  na.radius = (const double*)d_rad;
  na.M = (const int64_t*)d_M;
  na.weight = (const double2*)d_w;
  na.h = L.h;
  na.phihat_cheb = (const double*)d_cheb;
  na.cheb_deg = cdeg;
  na.tmax = smax * (1.0 + 1e-9);
  na.Kx = Kx;
  na.Ky = Ky;
  na.sx = sx;
  na.sy = sy;
  na.wt = wt;
  na.beta_t = beta_t;
  na.L1x = fx.store_L1; na.L2x = fx.store_L2; na.L1y = fy.store_L1; na.L2y = fy.store_L2;
  na.grid = (double2*)d_fine;
  int rc = launch_node_gather(na, (int)radius.size(), st);
  // inverse transform of the fine grid (storage order in, natural order out)
  if (!rc) rc = fft_cols<double>((double2*)d_fine, Kx, Kx, 1, 0, fy, +1, INT64_MAX, INT64_MAX, nullptr, 0, 16, st);
  if (!rc) rc = fft_rows<double>((double2*)d_fine, Ky, Kx, 1, 0, fx, +1, INT64_MAX, INT64_MAX, st);
  if (!rc) rc = launch_embed_symbol((const double2*)d_fine, Kx, Ky, sx, sy, (const double*)d_ipx, (const double*)d_ipy,
                                    L.nx, L.ny, (double2*)d_emb, L.Mx, L.My, st);
  // forward transform of the windowed H on the apply's FFT sizes
  if (!rc) rc = fft_rows<double>((double2*)d_emb, L.My, L.Mx, 1, 0, ex, -1, INT64_MAX, INT64_MAX, st);
  if (!rc) rc = fft_cols<double>((double2*)d_emb, L.Mx, L.Mx, 1, 0, ey, -1, INT64_MAX, INT64_MAX, nullptr, 0, 16, st);
  if (!rc && P.cc.id >= 0) {
    // column layout [kx <= Mx/2][ky <= My/2] for the compiled column convolution (the symbol of
    // a radial kernel on the symmetric grid window is even along both axes)
    P.symbol_complex = P.kind == 1 ? 1 : 0;
    const int64_t ncols = L.Mx / 2 + 1;  // even in kx as well: columns kx > Mx/2 read Mx - kx
    size_t sb = (size_t)ncols * (L.My / 2 + 1) * sizeof(T) * (P.symbol_complex ? 2 : 1);
    if (P.alloc(&P.symbol, sb) != hipSuccess) {
      freeall();
      return fail(SBD_ENOMEM, "symbol allocation failed");
    }
    rc = store_symbol_cols<T>((const double2*)d_emb, L.Mx, L.My, ncols, ex.store_L1, ex.store_L2, ey.store_L1,
                              ey.store_L2, 1.0 / ((double)L.Mx * (double)L.My), P.symbol_complex, P.symbol, st);
  } else if (!rc) {
    SymbolRemap r{L.Mx, L.My, ex.store_L1, ex.store_L2, ey.store_L1, ey.store_L2,
                  P.apx.store_L1, P.apx.store_L2, P.apy.store_L1, P.apy.store_L2};
    P.symbol_complex = P.kind == 1 ? 1 : 0;
    size_t sb = (size_t)L.Mx * L.My * sizeof(T) * (P.symbol_complex ? 2 : 1);
    if (P.alloc(&P.symbol, sb) != hipSuccess) {
      freeall();
      return fail(SBD_ENOMEM, "symbol allocation failed");
    }
    rc = launch_store_symbol<T>((const double2*)d_emb, r, 1.0 / ((double)L.Mx * (double)L.My), P.symbol_complex,
                                P.symbol, st);
  }
  hipError_t se = hipStreamSynchronize(st);
  freeall();
  if (rc || se != hipSuccess) return fail(SBD_EHIP, std::string("grid symbol kernels failed: ") + hipGetErrorString(se));
  return SBD_OK;
}

template <typename T>
sbd_status plan_device(Plan& P, const double* pts, const double* tpts, hipStream_t st) {
  Layout& L = P.L;
  const int64_t n = P.n;       // sources
  const int64_t m = P.n_tgt;   // targets (= sources for a single point set)
  const bool bip = P.bipartite != 0;
  // ---- binning: keys, counting sort by key, stable within keys
  int32_t *keys = nullptr, *counts = nullptr, *cstart = nullptr, *fill = nullptr, *tcstart = nullptr;
  int* flags = nullptr;
  double2 *xs = nullptr, *xt = nullptr;
  std::vector<void*> tmp;
  auto freetmp = [&] { for (void* q : tmp) dev_free(q); tmp.clear(); };
  auto talloc = [&](void** q, size_t b) {
    hipError_t e = dev_malloc(q, b);
    if (e == hipSuccess) tmp.push_back(*q);
    return e == hipSuccess;
  };
  const int64_t nm = std::max(n, m);
  if (!talloc((void**)&keys, nm * 4) || !talloc((void**)&counts, (L.nkeys + 1) * 4) ||
      !talloc((void**)&cstart, (L.nkeys + 1) * 4) || !talloc((void**)&fill, (L.nkeys + 1) * 4) ||
      !talloc((void**)&flags, 16) || !talloc((void**)&xs, n * sizeof(double2))) {
    freetmp();
    return fail(SBD_ENOMEM, "plan temporaries");
  }
  if (P.alloc((void**)&P.perm, n * 4) || P.alloc((void**)&P.skeys, n * 4) ||
      P.alloc(&P.loc, n * sizeof(cplx<T>)) || P.alloc((void**)&P.tile_start, (L.ntx * L.nty + 1) * 4) ||
      P.alloc((void**)&P.row_ptr, (m + 1) * 8)) {
    freetmp();
    return fail(SBD_ENOMEM, "plan arrays");
  }
  int hflags[4] = {0, 0, 0, 0};
  // sorts one point set: perm (sorted -> input), skeys, loc, sorted FP64 coordinates,
  // device cell starts and their host copy
  auto bin_set = [&](const double* p, int64_t cnt, int32_t* perm, int32_t* skeys, void* loc, double2* xsorted,
                     int32_t* cs, std::vector<int32_t>& hs) -> sbd_status {
    Layout Ls = L;
    Ls.n = cnt;
    if (hipMemsetAsync(counts, 0, (L.nkeys + 1) * 4, st) || hipMemsetAsync(fill, 0, (L.nkeys + 1) * 4, st) ||
        hipMemsetAsync(flags, 0, 16, st))
      return fail(SBD_EHIP, "memset");
    if (launch_keys(p, Ls, keys, counts, flags, st)) return fail(SBD_EHIP, "keys kernel");
    std::vector<int32_t> hc(L.nkeys + 1);
    if (hipMemcpyAsync(hc.data(), counts, (L.nkeys + 1) * 4, hipMemcpyDeviceToHost, st) ||
        hipMemcpyAsync(hflags, flags, 16, hipMemcpyDeviceToHost, st) || hipStreamSynchronize(st))
      return fail(SBD_EHIP, "readback counts");
    if (hflags[0]) return fail(SBD_EINVAL, "non-finite point coordinates");
    hs.assign(L.nkeys + 1, 0);
    int64_t acc = 0;
    for (int64_t k = 0; k < L.nkeys; ++k) { hs[k] = (int32_t)acc; acc += hc[k]; }
    hs[L.nkeys] = (int32_t)acc;
    if (hipMemcpyAsync(cs, hs.data(), (L.nkeys + 1) * 4, hipMemcpyHostToDevice, st))
      return fail(SBD_EHIP, "upload cell starts");
    if (launch_scatter(keys, cnt, cs, fill, perm, st) || launch_sort_cells(cs, L.nkeys, perm, st) ||
        launch_gather_sorted<T>(p, perm, Ls, xsorted, (cplx<T>*)loc, skeys, keys, st))
      return fail(SBD_EHIP, "binning kernels");
    return SBD_OK;
  };
  std::vector<int32_t> hs;
  const auto t_bin = std::chrono::steady_clock::now();
  sbd_status bs = bin_set(pts, n, P.perm, P.skeys, P.loc, xs, cstart, hs);
  if (bs != SBD_OK) { freetmp(); return bs; }
  const int64_t nt_tiles = L.ntx * L.nty;
  const int64_t ns2 = (int64_t)L.nsub * L.nsub;
  std::vector<int32_t> ts(nt_tiles + 1);
  for (int64_t t = 0; t <= nt_tiles; ++t) ts[t] = hs[t * ns2];
  if (hipMemcpyAsync(P.tile_start, ts.data(), ts.size() * 4, hipMemcpyHostToDevice, st)) {
    freetmp();
    return fail(SBD_EHIP, "upload tile starts");
  }
  // targets: the same layout, their own order
  std::vector<int32_t> tts = ts;
  if (bip) {
    std::vector<int32_t> hst;
    if (!talloc((void**)&xt, m * sizeof(double2)) || !talloc((void**)&tcstart, (L.nkeys + 1) * 4) ||
        P.alloc((void**)&P.tperm, m * 4) || P.alloc((void**)&P.tskeys, m * 4) || P.alloc(&P.tloc, m * sizeof(cplx<T>))) {
      freetmp();
      return fail(SBD_ENOMEM, "target arrays");
    }
    bs = bin_set(tpts, m, P.tperm, P.tskeys, P.tloc, xt, tcstart, hst);
    if (bs != SBD_OK) { freetmp(); return bs; }
    for (int64_t t = 0; t <= nt_tiles; ++t) tts[t] = hst[t * ns2];
  } else {
    xt = xs;
    P.tperm = P.perm;
    P.tskeys = P.skeys;
    P.tloc = P.loc;
  }
  // ---- pair set (fixed-radius neighbour search) and close-correction values
  int32_t* rcount = nullptr;
  if (!talloc((void**)&rcount, m * 4)) { freetmp(); return fail(SBD_ENOMEM, "row counts"); }
  const auto t_near = std::chrono::steady_clock::now();
  P.bin_seconds = std::chrono::duration<double>(t_near - t_bin).count();
  if (hipMemsetAsync(flags, 0, 16, st) ||
      launch_near_count(xt, P.tskeys, m, xs, cstart, L, P.d2max, bip ? 0 : 1, rcount, flags + 1, st)) {
    freetmp();
    return fail(SBD_EHIP, "near count");
  }
  std::vector<int32_t> rc(m);
  if (hipMemcpyAsync(rc.data(), rcount, m * 4, hipMemcpyDeviceToHost, st) ||
      hipMemcpyAsync(hflags, flags, 16, hipMemcpyDeviceToHost, st) || hipStreamSynchronize(st)) {
    freetmp();
    return fail(SBD_EHIP, "readback row counts");
  }
  if (hflags[1]) { freetmp(); return fail(SBD_EDUP, bip ? "a target coincides with a source" : "two distinct points coincide"); }
  std::vector<int64_t> rp(m + 1);
  rp[0] = 0;
  for (int64_t i = 0; i < m; ++i) rp[i + 1] = rp[i] + rc[i];
  P.nnz = rp[m];
  if (P.nnz >= (int64_t)INT32_MAX) { freetmp(); return fail(SBD_EUNSUPPORTED, "more than 2^31 close pairs"); }
  {
    // work units: split each non-empty tile into runs of at most kUnitMaxPoints points and
    // about kUnitNnz close entries (at least kUnitMinPoints points)
    std::vector<int32_t> ut, us;
    for (int64_t t = 0; t < nt_tiles; ++t) {
      int64_t p = tts[t];
      const int64_t e = tts[t + 1];
      while (p < e) {
        int64_t q = std::min<int64_t>(e, p + kUnitMaxPoints);
        if (rp[q] - rp[p] > kUnitNnz) {
          // smallest q' in (p, q] with rp[q'] - rp[p] > kUnitNnz, then step back one row
          int64_t lo = p + 1, hi = q;
          while (lo < hi) {
            int64_t mid = (lo + hi) / 2;
            if (rp[mid] - rp[p] > kUnitNnz) hi = mid; else lo = mid + 1;
          }
          q = std::max<int64_t>(std::min<int64_t>(e, p + kUnitMinPoints), lo - 1);
          q = std::min<int64_t>(q, std::min<int64_t>(e, p + kUnitMaxPoints));
          if (q <= p) q = p + 1;
        }
        ut.push_back((int32_t)t);
        us.push_back((int32_t)p);
        p = q;
      }
    }
    us.push_back((int32_t)m);
    P.nunits = (int64_t)ut.size();
    if (P.alloc((void**)&P.unit_tile, std::max<size_t>(1, ut.size()) * 4) || P.alloc((void**)&P.unit_start, us.size() * 4) ||
        (P.nunits && hipMemcpyAsync(P.unit_tile, ut.data(), ut.size() * 4, hipMemcpyHostToDevice, st)) ||
        hipMemcpyAsync(P.unit_start, us.data(), us.size() * 4, hipMemcpyHostToDevice, st) ||
        hipStreamSynchronize(st)) {
      freetmp();
      return fail(SBD_EHIP, "work units");
    }
  }
  if (P.alloc((void**)&P.col, P.nnz * 4) || P.alloc((void**)&P.val, P.nnz * 8)) {
    freetmp();
    return fail(SBD_ENOMEM, "CSR arrays");
  }
  // a general kernel's tables are in r; their degree grows with the oscillation over [0, delta_min]
  int deg = 28;
  if (P.general) {
    double fr = 0.0;
    for (const TrigTerm& t : P.gk.terms) fr = std::max(fr, t.w);
    for (int p = 0; p < P.fit.P; ++p) fr = std::max(fr, P.fit.radii[p] / P.delta_max);
    deg = std::min(96, std::max(28, 28 + (int)std::ceil(0.5 * fr * P.delta_min)));
  }
  NearTables nt = near_tables(P.fit, P.general ? 2 : P.kind, P.delta_max, P.d2max, P.wavenumber, deg,
                              P.general ? &P.gk : nullptr);
  P.self_im = nt.self.imag();
  double *dA = nullptr, *dB = nullptr;
  if (!talloc((void**)&dA, (deg + 1) * 8) || !talloc((void**)&dB, (deg + 1) * 8)) {
    freetmp();
    return fail(SBD_ENOMEM, "tables");
  }
  if (hipMemcpyAsync(P.row_ptr, rp.data(), (m + 1) * 8, hipMemcpyHostToDevice, st) ||
      hipMemcpyAsync(dA, nt.A.data(), (deg + 1) * 8, hipMemcpyHostToDevice, st) ||
      hipMemcpyAsync(dB, nt.B.data(), (deg + 1) * 8, hipMemcpyHostToDevice, st) ||
      launch_near_fill(xt, P.tskeys, m, xs, cstart, L, P.d2max, bip ? 0 : 1, P.row_ptr, P.col, P.val, dA, dB, deg,
                       P.d2max, nt.self.real(), P.general ? 1 : 0, st) ||
      hipStreamSynchronize(st)) {
    freetmp();
    return fail(SBD_EHIP, "near fill");
  }
  const auto t_fill = std::chrono::steady_clock::now();
  P.near_seconds = std::chrono::duration<double>(t_fill - t_near).count();
  if (P.near_assembly) {
    sbd_status as = assemble_pairdiff(P, xt, xs, st);
    if (as != SBD_OK) { freetmp(); return as; }
    P.assembly_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_fill).count();
  }
  freetmp();
  if (!P.precision && P.near_fp32) {
    // D rounded to FP32 (relative rounding 6e-8 per entry, far below the FP32 far field's
    // error), rows summed in FP32; the FP64 entries are released
    if (P.alloc((void**)&P.valf, P.nnz * 4)) return fail(SBD_ENOMEM, "CSR values (FP32)");
    if (launch_to_f32(P.val, P.valf, P.nnz, st) || hipStreamSynchronize(st) != hipSuccess)
      return fail(SBD_EHIP, "CSR values (FP32)");
    P.release(P.val, P.nnz * 8);
    P.val = nullptr;
  }
  return SBD_OK;
}

}  // namespace

namespace {

// Workspace of sbd_apply_noalloc: one static array per device, held until the process
// ends.  In host code `scratch` is a host-side stand-in, never a device address: the
// device address comes from hipGetSymbolAddress, once per device, and only that address
// is handed to kernels.
__device__ __align__(256) unsigned char scratch[SBD_NOALLOC_SCRATCH_BYTES];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

sbd_status scratch_address(void** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
    return fail(SBD_EHIP, "sbd_apply_noalloc: no current HIP device");
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(SBD_EHIP, std::string("sbd_apply_noalloc: hipGetSymbolAddress(scratch) failed: ") +
                                hipGetErrorString(e));
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return SBD_OK;
}

template <typename T>
sbd_status apply_t(Plan& P, const void* f, void* q, int nrhs, int dtype, int parts, void* ws, hipStream_t st) {
  const Layout& L = P.L;
  WsLayout wl = ws_layout(P, nrhs);
  char* base = (char*)ws;
  ApplyArgs a;
  a.Ld = &L;
  a.n = P.n;
  a.nrhs = nrhs;
  a.in_dtype = dtype;
  a.cplx_data = (dtype == SBD_C128 || dtype == SBD_C64) ? 1 : 0;
  a.f = f;
  a.q = q;
  a.perm = P.perm;
  a.tile_start = P.tile_start;
  a.nt = P.n_tgt;
  a.tperm = P.tperm;
  a.tloc = P.tloc;
  a.self = P.bipartite ? 0 : 1;
  a.unit_tile = P.unit_tile;
  a.unit_start = P.unit_start;
  a.nunits = P.nunits;
  a.loc = P.loc;
  a.ntiles = L.ntx * L.nty;
  a.T = L.T;
  a.w = L.w;
  a.PL = L.PL;
  a.SG = L.SG;
  a.beta = L.beta;
  a.ntx = L.ntx;
  a.sub = base;
  a.grid = base + wl.sub;
  a.fs = base + wl.sub + wl.grid;
  a.Mx = L.Mx;
  a.My = L.My;
  a.nx = L.nx;
  a.ny = L.ny;
  a.row_ptr = P.row_ptr;
  a.col = P.col;
  a.val = P.valf ? (const void*)P.valf : (const void*)P.val;
  a.val_f32 = P.valf ? 1 : 0;
  a.deterministic = P.deterministic;
  a.sorted_io = (parts & SBD_IO_SORTED) ? 1 : 0;
  a.self_im = P.self_im;
  a.parts = parts & SBD_PART_ALL;
  a.nnz = P.nnz;
  {
    double mean = (double)P.nnz / (double)std::max<int64_t>(1, P.n_tgt);
    int G = 1;
    while (G < 64 && G < mean) G *= 2;
    a.csr_group = G;
  }
  a.real_grid = (!a.cplx_data && P.real_rows) ? 1 : 0;
  // several right-hand sides: the close correction of all of them in one pass over D (the
  // sorted f copy interleaved per point), added by the interpolation
  const bool multi_near = nrhs > 1 && nrhs <= 64 && (parts & SBD_PART_NEAR);
  a.fs_inter = multi_near ? 1 : 0;
  a.qnear = nullptr;
  if (launch_spread<T>(a, st)) return fail(SBD_EHIP, "spread launch");
  if (multi_near) {
    a.qnear = base + wl.sub + wl.grid + wl.fs;
    if (launch_near_multi<T>(a, st)) return fail(SBD_EHIP, "close-correction launch");
  }
  if ((parts & SBD_PART_FAR) && a.real_grid) {
    cplx<T>* g = (cplx<T>*)a.grid;
    int64_t sb = L.Mx * L.My;
    RealRowArgs ra;
    ra.ny = L.ny;
    ra.nx = L.nx;
    ra.M = L.Mx;
    ra.gpitch = L.Mx;
    ra.nbatch = nrhs;
    ra.sbatch = sb;
    ra.sub = a.sub;
    ra.T = L.T;
    ra.SG = L.SG;
    ra.log2T = 0;
    while ((1 << ra.log2T) < L.T) ++ra.log2T;
    ra.ntx = L.ntx;
    ra.nty = L.nty;
    ra.ntiles = L.ntx * L.nty;
    // compiled rows and columns: the spectra interleaved in row pairs, so the column pass
    // reads and writes two rows per access; the inverse rows take two rows per workgroup
    ra.pair = (P.row_pairs && P.rr.id >= 0 && P.cc.id >= 0 && P.rr.pairs) ? 1 : 0;
    if (P.rr.id >= 0 ? rows_r2c_cc<T>(g, ra, P.rr, st) : rows_r2c<T>(g, ra, P.rrp, st))
      return fail(SBD_EHIP, "real row FFT launch");
    if (P.cc.id >= 0) {
      if (colconv<T>(g, L.Mx / 2 + 1, L.Mx, nrhs, sb, P.cc, L.ny, L.ny, P.symbol, P.symbol_complex, L.Mx,
                     ra.pair ? 2 : 1, st))
        return fail(SBD_EHIP, "column convolution launch");
    } else if (fft_cols<T>(g, L.Mx / 2 + 1, L.Mx, nrhs, sb, P.apy, -1, L.ny, L.ny, P.symbol, P.symbol_complex, 16, st))
      return fail(SBD_EHIP, "column FFT launch");
    if (P.rr.id >= 0 ? rows_c2r_cc<T>(g, ra, P.rr, st) : rows_c2r<T>(g, ra, P.rrp, st))
      return fail(SBD_EHIP, "inverse real row FFT launch");
  } else if (parts & SBD_PART_FAR) {
    if (launch_gather_grid<T>(a, st)) return fail(SBD_EHIP, "grid assembly launch");
    cplx<T>* g = (cplx<T>*)a.grid;
    int64_t sb = L.Mx * L.My;
    if (fft_rows<T>(g, L.ny, L.Mx, nrhs, sb, P.apx, -1, L.nx, INT64_MAX, st))
      return fail(SBD_EHIP, "row FFT launch");
    if (P.cc.id >= 0) {
      if (colconv<T>(g, L.Mx, L.Mx, nrhs, sb, P.cc, L.ny, L.ny, P.symbol, P.symbol_complex, L.Mx, 1, st))
        return fail(SBD_EHIP, "column convolution launch");
    } else if (fft_cols<T>(g, L.Mx, L.Mx, nrhs, sb, P.apy, -1, L.ny, L.ny, P.symbol, P.symbol_complex, 16, st))
      return fail(SBD_EHIP, "column FFT launch");
    if (fft_rows<T>(g, L.ny, L.Mx, nrhs, sb, P.apx, +1, INT64_MAX, L.nx, st))
      return fail(SBD_EHIP, "inverse row FFT launch");
  }
  if (launch_interp_near<T>(a, st)) return fail(SBD_EHIP, "interpolation launch");
  return SBD_OK;
}

}  // namespace
}  // namespace sbd

using namespace sbd;

extern "C" {

void sbd_default_options(sbd_options* opt) {
  if (!opt) return;
  std::memset(opt, 0, sizeof(*opt));
  opt->delta_min = 0.0;
  opt->precision = 0;
  opt->max_rhs = 1;
  opt->nufft_tol = 0.0;
  opt->sigma = 0.0;
  opt->force_order = 0;
  opt->tile = 0;
  opt->byte_cap = 0;
  opt->fit_reuse = 0;
}

const char* sbd_strerror(sbd_status s) {
  switch (s) {
    case SBD_OK: return "ok";
    case SBD_EINVAL: return "invalid argument";
    case SBD_ENOMEM: return "out of memory";
    case SBD_EDUP: return "coincident points";
    case SBD_ENOCONV: return "iteration stopped before reaching the tolerance";
    case SBD_EFLOOR: return "tolerance below the SBD floor";
    case SBD_EHIP: return "HIP runtime error";
    case SBD_EUNSUPPORTED: return "unsupported";
  }
  return "unknown status";
}

const char* sbd_last_error(void) { return g_last_error.c_str(); }

static sbd_status plan_impl(const double* points, int64_t n, const double* targets, int64_t m, bool bip,
                            const sbd_kernel* kernel, double eps, const sbd_options* opt_in, void* stream,
                            sbd_plan_t* out) {
  if (!out) return fail(SBD_EINVAL, "out is NULL");
  *out = nullptr;
  g_last_error.clear();
  auto t0 = std::chrono::steady_clock::now();
  if (!points || n < (bip ? 1 : 2) || !kernel || !(eps > 0) || !(eps < 1))
    return fail(SBD_EINVAL, bip ? "need sources, n >= 1, 0 < eps < 1" : "need points, n >= 2, 0 < eps < 1");
  if (bip && (!targets || m < 1)) return fail(SBD_EINVAL, "need targets, m >= 1");
  if (n >= (int64_t)INT32_MAX || m >= (int64_t)INT32_MAX) return fail(SBD_EUNSUPPORTED, "n or m >= 2^31");
  if (kernel->kind != SBD_LAPLACE && kernel->kind != SBD_HELMHOLTZ && kernel->kind != SBD_GENERAL)
    return fail(SBD_EINVAL, "unknown kernel");
  if (kernel->kind == SBD_HELMHOLTZ && !(kernel->wavenumber > 0)) return fail(SBD_EINVAL, "wavenumber must be > 0");
  GeneralKernel gk;
  if (kernel->kind == SBD_GENERAL) {
    if (kernel->nterms < 0 || kernel->nterms > 8 || (kernel->nterms && !kernel->terms))
      return fail(SBD_EINVAL, "general kernel: need 0 <= nterms <= 8 and terms");
    if (kernel->enforce < 0 || kernel->enforce > 4) return fail(SBD_EINVAL, "general kernel: need 0 <= enforce <= 4");
    if (!std::isfinite(kernel->c_log)) return fail(SBD_EINVAL, "general kernel: c_log not finite");
    gk.c_log = kernel->c_log;
    gk.enforce = kernel->enforce;
    for (int j = 0; j < kernel->nterms; ++j) {
      const double* t = kernel->terms + 4 * j;
      if (!(t[0] >= 0 && t[0] <= 8 && t[0] == std::floor(t[0])) || !(t[1] >= 0) || !std::isfinite(t[1]) ||
          !std::isfinite(t[2]) || !std::isfinite(t[3]))
        return fail(SBD_EINVAL, "general kernel: each term needs an integer m in [0, 8], finite w >= 0, a, b");
      gk.terms.push_back(TrigTerm{(int)t[0], t[1], t[2], t[3]});
    }
    if (gk.c_log == 0.0 && gk.terms.empty()) return fail(SBD_EINVAL, "general kernel: G is zero");
  }
  sbd_options opt;
  sbd_default_options(&opt);
  if (opt_in) opt = *opt_in;
  if (opt.max_rhs < 1) opt.max_rhs = 1;
  hipStream_t st = (hipStream_t)stream;
  // plan memory and temporaries are stream-ordered on the plan's stream (no device-wide
  // synchronisation while planning)
  AllocStream alloc_scope(st);
  auto P = new Plan();
  if (hipGetDevice(&P->device) != hipSuccess) P->device = 0;
  P->n = n;
  P->n_tgt = bip ? m : n;
  P->bipartite = bip ? 1 : 0;
  P->general = kernel->kind == SBD_GENERAL;
  P->kind = P->general ? (int)SBD_LAPLACE : kernel->kind;
  P->gk = gk;
  P->wavenumber = kernel->kind == SBD_HELMHOLTZ ? kernel->wavenumber : 0.0;
  P->precision = opt.precision ? 1 : 0;
  P->max_rhs = opt.max_rhs;
  P->eps = eps;
  P->byte_cap = opt.byte_cap;
  P->timing = opt.timing ? 1 : 0;
  P->near_fp32 = (opt.near_fp32 && !opt.precision) ? 1 : 0;
  P->deterministic = opt.deterministic ? 1 : 0;
  if (opt.near_assembly != 0 && opt.near_assembly != 1) {
    delete P;
    return fail(SBD_EINVAL, "near_assembly must be 0 or 1");
  }
  P->near_assembly = opt.near_assembly;
  auto bail = [&](sbd_status s) { delete P; return s; };
  // ---- geometry (bounding-box centre, delta_max = 2 max |z - c|)
  // (over sources and targets together)
  const int nb = (int)std::min<int64_t>(1024, std::max<int64_t>(1, ceil_div(std::max(n, P->n_tgt), 256)));
  double* part = nullptr;
  if (dev_malloc((void**)&part, nb * 4 * sizeof(double))) return bail(fail(SBD_ENOMEM, "partials"));
  std::vector<double> hp(nb * 4);
  double mnx = INFINITY, mny = INFINITY, mxx = -INFINITY, mxy = -INFINITY;
  for (int set = 0; set < (bip ? 2 : 1); ++set) {
    const double* ps = set ? targets : points;
    const int64_t cnt = set ? m : n;
    if (launch_bbox_partials(ps, cnt, part, nb, st) ||
        hipMemcpyAsync(hp.data(), part, nb * 4 * sizeof(double), hipMemcpyDeviceToHost, st) ||
        hipStreamSynchronize(st)) {
      dev_free(part);
      return bail(fail(SBD_EHIP, std::string("bbox: ") + hipGetErrorString(hipGetLastError())));
    }
    for (int b = 0; b < nb; ++b) {
      mnx = std::min(mnx, hp[4 * b]); mny = std::min(mny, hp[4 * b + 1]);
      mxx = std::max(mxx, hp[4 * b + 2]); mxy = std::max(mxy, hp[4 * b + 3]);
    }
  }
  if (!std::isfinite(mnx) || !std::isfinite(mxx) || !std::isfinite(mny) || !std::isfinite(mxy)) {
    dev_free(part);
    return bail(fail(SBD_EINVAL, "non-finite coordinates"));
  }
  P->cx = 0.5 * (mnx + mxx);
  P->cy = 0.5 * (mny + mxy);
  double r2 = 0;
  for (int set = 0; set < (bip ? 2 : 1); ++set) {
    const double* ps = set ? targets : points;
    const int64_t cnt = set ? m : n;
    if (launch_radius_partials(ps, cnt, P->cx, P->cy, part, nb, st) ||
        hipMemcpyAsync(hp.data(), part, nb * sizeof(double), hipMemcpyDeviceToHost, st) || hipStreamSynchronize(st)) {
      dev_free(part);
      return bail(fail(SBD_EHIP, "radius"));
    }
    for (int b = 0; b < nb; ++b) r2 = std::max(r2, hp[b]);
  }
  dev_free(part);
  P->delta_max = 2.0 * std::sqrt(r2);
  if (!(P->delta_max > 0)) return bail(fail(SBD_EINVAL, "all points coincide"));
  if (opt.delta_min > 0) P->delta_min = opt.delta_min;
  else P->delta_min = std::pow(std::fabs(std::log(eps)), 2.0 / 3.0) / std::pow((double)n, 2.0 / 3.0) * P->delta_max;
  double a = P->delta_min / P->delta_max;
  if (!(a > 0 && a < 1)) return bail(fail(SBD_EINVAL, "need 0 < delta_min < delta_max"));
  // ---- SBD fit (host FP64)
  auto tf = std::chrono::steady_clock::now();
  std::string msg;
  int nth = (int)std::min<unsigned>(16, std::max(1u, std::thread::hardware_concurrency()));
  int frc = P->general ? sbd_fit_general(P->gk, P->delta_max, a, eps, nth, P->fit, msg)
                       : cached_fit(P->kind, a, eps, P->kind == 1 ? P->wavenumber * P->delta_max : 0.0,
                                    opt.force_order, nth, opt.fit_reuse != 0, P->fit, msg);
  P->fit_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - tf).count();
  if (frc) return bail(fail((sbd_status)frc, msg));
  // ---- NUFFT parameters
  double tol = opt.nufft_tol > 0 ? opt.nufft_tol : eps;
  double tolfloor = P->precision ? 1e-14 : 2e-8;
  tol = std::max(tol, tolfloor);
  P->nufft_tol = tol;
  P->pd_tol = std::max(1e-13, std::min(1e-8, 1e-3 * tol));
  double sigma, beta;
  int w;
  es_params(opt.sigma > 0 ? opt.sigma : 1.25, tol, &sigma, &w, &beta);
  P->sigma = sigma;
  double S = *std::max_element(P->fit.radii.begin(), P->fit.radii.end()) / P->delta_max;
  if (P->kind == 1) S = std::max(S, P->wavenumber);
  Layout& L = P->L;
  L.n = n;
  L.h = kPi / (sigma * S);
  L.inv_h = 1.0 / L.h;
  L.w = w;
  L.beta = beta;
  L.PL = (w + 1) / 2;
  {
    // tile edge: power of two, covers the kernel pad, fine cells at least delta_min wide,
    // one padded tile in the LDS of the spread and interpolation workgroups
    std::string lmsg;
    int lrc = choose_tile(opt.tile, w, L.h, P->delta_min, P->precision, max_lds(), kUnitPoints, &L.T, lmsg);
    if (lrc) return bail(fail((sbd_status)lrc, lmsg));
  }
  L.SG = L.T + 2 * L.PL;
  L.x0 = mnx;
  L.y0 = mny;
  double tileh = L.T * L.h;
  L.nsub = std::max(1, (int)std::floor(tileh / (P->delta_min * (1.0 + 1e-9))));
  if (L.nsub > 64) L.nsub = 64;
  L.inv_c = (double)L.nsub / tileh;
  int64_t ncx = (int64_t)std::floor((mxx - L.x0) * L.inv_c) + 1;
  int64_t ncy = (int64_t)std::floor((mxy - L.y0) * L.inv_c) + 1;
  L.ntx = ceil_div(ncx, L.nsub);
  L.nty = ceil_div(ncy, L.nsub);
  L.ncx = L.ntx * L.nsub;
  L.ncy = L.nty * L.nsub;
  L.nkeys = L.ntx * L.nty * (int64_t)L.nsub * L.nsub;
  if (L.nkeys >= (int64_t)INT32_MAX / 2) return bail(fail(SBD_EUNSUPPORTED, "too many near-field cells"));
  L.nx = L.ntx * L.T + 2 * L.PL;
  L.ny = L.nty * L.T + 2 * L.PL;
  const bool dbl = P->precision == 1;
  // Laplace rows are real: length Mx = 2 N with N >= nx, from the compiled real-row
  // transforms when one is within 15% of the generic size (SBD_COLCONV=0 keeps the
  // generic ones, read at plan time like the column choice below)
  const char* cc_env = getenv("SBD_COLCONV");
  const bool cc_allow = !cc_env || atoi(cc_env) != 0;
  const char* rp_env = getenv("SBD_ROW_PAIRS");
  P->row_pairs = (!rp_env || atoi(rp_env) != 0) ? 1 : 0;
  int64_t rrN = 0;
  if (P->kind == SBD_LAPLACE) {
    const int64_t g = best_fft_size(L.nx, 1, dbl);
    const int64_t c = cc_allow ? rows_size(L.nx, dbl) : 0;
    rrN = (c > 0 && (double)c <= 1.15 * (double)g) ? c : 0;
    L.Mx = 2 * (rrN ? rrN : g);
  } else {
    L.Mx = best_fft_size(2 * L.nx - 1, 1, dbl);
  }
  P->d2max = P->delta_min * P->delta_min;
  if (build_axis_plan(P->apx, L.Mx, dbl, max_lds(), 1)) return bail(fail(SBD_ENOMEM, "FFT axis plans"));
  if (P->kind == SBD_LAPLACE && !P->apx.four_step) {
    if (rrN) {
      if (build_row_plan(P->rr, rrN, dbl) != 0) return bail(fail(SBD_ENOMEM, "row transform tables"));
      P->real_rows = 1;
    } else if (build_real_row_plan(P->rrp, L.Mx, dbl, max_lds()) == 0) {
      P->real_rows = 1;
    }
  }
  {
    // Column length: the compiled whole-column convolution's smallest length >= 2 ny - 1
    // when it exceeds the generic transform's size by at most 15% (it runs about twice as
    // fast per element), else the generic column passes.  It needs the row transforms to
    // leave the spectrum in natural order (no four-step rows).  SBD_COLCONV=0 keeps the
    // generic passes; it is read at plan time, since the symbol layout follows the choice.
    // Complex f on a Laplace plan uses the complex grid, whose columns the same kernel takes.
    const int64_t need = 2 * L.ny - 1;
    const int64_t generic = best_fft_size(need, 1, dbl);
    const bool allow = cc_allow && !P->apx.four_step;
    const bool ch = P->kind == SBD_HELMHOLTZ;
    const int64_t ccl = allow ? colconv_size(need, dbl, ch) : 0;
    if (ccl > 0 && (double)ccl <= 1.15 * (double)generic) {
      L.My = ccl;
      if (build_colconv_plan(P->cc, L.My, dbl, ch) != 0) return bail(fail(SBD_ENOMEM, "column convolution tables"));
    } else {
      L.My = generic;
      if (build_axis_plan(P->apy, L.My, dbl, max_lds(), 16)) return bail(fail(SBD_ENOMEM, "FFT axis plans"));
    }
  }
  // The Toeplitz symbol needs only the layout and the fit: a second host thread builds it on
  // a stream of its own while this thread bins the points and assembles the close
  // correction (the node spreading and transforms overlap the neighbour search on the GPU).
  int dev = 0;
  hipStream_t sym_st = nullptr;
  if (hipGetDevice(&dev) != hipSuccess || hipStreamCreateWithFlags(&sym_st, hipStreamNonBlocking) != hipSuccess)
    return bail(fail(SBD_EHIP, "symbol stream"));
  sbd_status sym_status = SBD_OK;
  std::string sym_msg;
  std::thread sym_thread([&] {
    (void)hipSetDevice(dev);
    AllocStream sym_scope(sym_st);
    const auto t_sym = std::chrono::steady_clock::now();
    sym_status = dbl ? build_symbol<double>(*P, sym_st) : build_symbol<float>(*P, sym_st);
    if (sym_status != SBD_OK) sym_msg = sbd_last_error();
    P->symbol_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_sym).count();
  });
  sbd_status s = dbl ? plan_device<double>(*P, points, bip ? targets : points, st)
                     : plan_device<float>(*P, points, bip ? targets : points, st);
  sym_thread.join();
  (void)hipStreamSynchronize(sym_st);
  (void)hipStreamDestroy(sym_st);
  if (s != SBD_OK) return bail(s);
  if (sym_status != SBD_OK) return bail(fail(sym_status, sym_msg));
  if (P->byte_cap && P->resident + ws_layout(*P, P->max_rhs).total > P->byte_cap)
    return bail(fail(SBD_ENOMEM, "plan and workspace exceed byte_cap"));
  P->plan_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  *out = reinterpret_cast<sbd_plan_t>(P);
  return SBD_OK;
}

sbd_status sbd_set_cache_limit(size_t bytes) {
  std::lock_guard<std::mutex> g(g_cache_mu);
  g_cache_limit = bytes;
  cache_trim(bytes);
  return SBD_OK;
}

size_t sbd_cache_bytes(void) {
  std::lock_guard<std::mutex> g(g_cache_mu);
  return g_cache_held;
}

sbd_status sbd_prefit(const sbd_kernel* kernel, double eps, double a, double delta_max, int force_order,
                      int* out_P) {
  g_last_error.clear();
  if (!kernel) return fail(SBD_EINVAL, "kernel is NULL");
  if (kernel->kind == SBD_GENERAL)
    return fail(SBD_EUNSUPPORTED, "sbd_prefit: SBD_LAPLACE and SBD_HELMHOLTZ only (general kernels are fitted per plan)");
  if (kernel->kind != SBD_LAPLACE && kernel->kind != SBD_HELMHOLTZ) return fail(SBD_EINVAL, "unknown kernel");
  if (kernel->kind == SBD_HELMHOLTZ && !(kernel->wavenumber > 0 && delta_max > 0))
    return fail(SBD_EINVAL, "sbd_prefit: Helmholtz needs wavenumber > 0 and delta_max > 0");
  if (!(eps > 0 && eps < 1) || !(a > 0 && a < 1)) return fail(SBD_EINVAL, "sbd_prefit: need 0 < eps < 1, 0 < a < 1");
  FitResult fr;
  std::string msg;
  const int nth = (int)std::min<unsigned>(16, std::max(1u, std::thread::hardware_concurrency()));
  const double kappa = kernel->kind == SBD_HELMHOLTZ ? kernel->wavenumber * delta_max : 0.0;
  int rc = cached_fit(kernel->kind, a, eps, kappa, force_order, nth, true, fr, msg);
  if (rc) return fail((sbd_status)rc, msg);
  if (out_P) *out_P = fr.P;
  return SBD_OK;
}

sbd_status sbd_plan(const double* points, int64_t n, const sbd_kernel* kernel, double eps, const sbd_options* opt,
                    void* stream, sbd_plan_t* out) {
  return plan_impl(points, n, nullptr, 0, false, kernel, eps, opt, stream, out);
}

sbd_status sbd_plan_targets(const double* targets, int64_t m, const double* sources, int64_t n,
                            const sbd_kernel* kernel, double eps, const sbd_options* opt, void* stream,
                            sbd_plan_t* out) {
  return plan_impl(sources, n, targets, m, true, kernel, eps, opt, stream, out);
}

size_t sbd_workspace_bytes(sbd_plan_t plan, int nrhs) {
  if (!plan || nrhs < 1) return 0;
  return ws_layout(*reinterpret_cast<Plan*>(plan), nrhs).total;
}

size_t sbd_plan_bytes(sbd_plan_t plan) {
  if (!plan) return 0;
  return reinterpret_cast<Plan*>(plan)->resident;
}


sbd_status sbd_apply_parts(sbd_plan_t plan, const void* f, void* q, int nrhs, int dtype, int parts, void* workspace,
                           size_t workspace_bytes, void* stream) {
  if (!plan || !f || !q) return fail(SBD_EINVAL, "NULL plan, f or q");
  Plan& P = *reinterpret_cast<Plan*>(plan);
  if (nrhs < 1 || nrhs > P.max_rhs) return fail(SBD_EINVAL, "nrhs outside [1, max_rhs]");
  if (dtype < 0 || dtype > 3) return fail(SBD_EINVAL, "bad dtype");
  if (P.kind == SBD_HELMHOLTZ && (dtype == SBD_F64 || dtype == SBD_F32))
    return fail(SBD_EINVAL, "Helmholtz needs complex f and q");
  if ((parts & SBD_PART_ALL) == 0) return fail(SBD_EINVAL, "parts selects nothing");
  if (parts & ~(SBD_PART_ALL | SBD_IO_SORTED)) return fail(SBD_EINVAL, "unknown parts bits");
  size_t need = ws_layout(P, nrhs).total;
  void* ws = workspace;
  if (ws) {
    if (workspace_bytes < need) return fail(SBD_EINVAL, "workspace too small");
  } else {
    if (!P.ws || P.ws_bytes < need) {
      AllocStream scope((hipStream_t)stream);  // ordered on the apply's stream
      if (P.ws) dev_free(P.ws);
      P.ws = nullptr;
      size_t full = ws_layout(P, P.max_rhs).total;
      if (dev_malloc(&P.ws, full) != hipSuccess) {
        P.ws = nullptr;
        P.ws_bytes = 0;
        return fail(SBD_ENOMEM, "workspace allocation");
      }
      P.ws_bytes = full;
    }
    ws = P.ws;
  }
  hipStream_t st = (hipStream_t)stream;
  if (P.timing) {
    g_marks = &P.marks;
    mark_launch("begin", st, 0.0);
    P.t_calls += 1;
  }
  sbd_status s = P.precision ? apply_t<double>(P, f, q, nrhs, dtype, parts, ws, st)
                             : apply_t<float>(P, f, q, nrhs, dtype, parts, ws, st);
  g_marks = nullptr;
  if (P.timing && P.marks.marks.size() > 4096) P.drain_marks();
  return s;
}

int sbd_set_timing(sbd_plan_t plan, int enable) {
  if (!plan) return -1;
  Plan& P = *reinterpret_cast<Plan*>(plan);
  P.drain_marks();
  P.timing = enable ? 1 : 0;
  return 0;
}

int sbd_launch_times(sbd_plan_t plan, char* names, size_t names_bytes, double* ms, double* bytes, int max_entries) {
  if (!plan) return -1;
  Plan& P = *reinterpret_cast<Plan*>(plan);
  P.drain_marks();
  std::string all;
  int n = 0;
  for (size_t k = 0; k < P.t_names.size() && n < max_entries; ++k, ++n) {
    if (ms) ms[n] = P.t_calls ? P.t_ms[k] / (double)P.t_calls : 0.0;
    if (bytes) bytes[n] = P.t_calls ? P.t_bytes[k] / (double)P.t_calls : 0.0;
    all += P.t_names[k] + "\n";
  }
  if (names && names_bytes) {
    size_t c = std::min(names_bytes - 1, all.size());
    std::memcpy(names, all.data(), c);
    names[c] = 0;
  }
  P.t_names.clear();
  P.t_ms.clear();
  P.t_bytes.clear();
  P.t_cnt.clear();
  P.t_calls = 0;
  return n;
}

sbd_status sbd_apply(sbd_plan_t plan, const void* f, void* q, int nrhs, int dtype, void* workspace,
                     size_t workspace_bytes, void* stream) {
  return sbd_apply_parts(plan, f, q, nrhs, dtype, SBD_PART_ALL, workspace, workspace_bytes, stream);
}

sbd_status sbd_apply_noalloc(sbd_plan_t plan, const void* f, void* q, int nrhs, int dtype, void* stream) {
  if (!plan || !f || !q) return fail(SBD_EINVAL, "NULL plan, f or q");
  Plan& P = *reinterpret_cast<Plan*>(plan);
  if (nrhs < 1 || nrhs > P.max_rhs) return fail(SBD_EINVAL, "nrhs outside [1, max_rhs]");
  if (dtype < 0 || dtype > 3) return fail(SBD_EINVAL, "bad dtype");
  if (P.kind == SBD_HELMHOLTZ && (dtype == SBD_F64 || dtype == SBD_F32))
    return fail(SBD_EINVAL, "Helmholtz needs complex f and q");
  const size_t need = ws_layout(P, nrhs).total;
  if (need > (size_t)SBD_NOALLOC_SCRATCH_BYTES)
    return fail(SBD_ENOMEM, "sbd_apply_noalloc: the apply needs " + std::to_string(need) +
                                " bytes of workspace, above the " + std::to_string((size_t)SBD_NOALLOC_SCRATCH_BYTES) +
                                "-byte static scratch (use sbd_apply with a workspace)");
  void* ws = nullptr;
  sbd_status s = scratch_address(&ws);
  if (s != SBD_OK) return s;
  // no launch marks (events) here: nothing is created or allocated on this path
  hipStream_t st = (hipStream_t)stream;
  return P.precision ? apply_t<double>(P, f, q, nrhs, dtype, SBD_PART_ALL, ws, st)
                     : apply_t<float>(P, f, q, nrhs, dtype, SBD_PART_ALL, ws, st);
}

sbd_status sbd_plan_info(sbd_plan_t plan, sbd_info* o) {
  if (!plan || !o) return fail(SBD_EINVAL, "NULL argument");
  const Plan& P = *reinterpret_cast<Plan*>(plan);
  std::memset(o, 0, sizeof(*o));
  o->n = P.n;
  o->n_targets = P.n_tgt;
  o->bipartite = P.bipartite;
  o->kind = P.general ? (int)SBD_GENERAL : P.kind;
  o->precision = P.precision;
  o->P = P.fit.P;
  o->n_xi = P.n_xi;
  o->nnz = P.nnz;
  o->eps = P.eps;
  o->delta_min = P.delta_min;
  o->delta_max = P.delta_max;
  o->center_x = P.cx;
  o->center_y = P.cy;
  o->fit_error = P.fit.err;
  o->h = P.L.h;
  o->w = P.L.w;
  o->beta = P.L.beta;
  o->sigma = P.sigma;
  o->nx = P.L.nx;
  o->ny = P.L.ny;
  o->Mx = P.L.Mx;
  o->My = P.L.My;
  o->tile = P.L.T;
  o->ntx = P.L.ntx;
  o->nty = P.L.nty;
  o->x0 = P.L.x0;
  o->y0 = P.L.y0;
  o->inv_c = P.L.inv_c;
  o->ncx = P.L.ncx;
  o->ncy = P.L.ncy;
  o->nsub = P.L.nsub;
  o->d2max = P.d2max;
  o->plan_seconds = P.plan_seconds;
  o->fit_seconds = P.fit_seconds;
  o->plan_bytes = P.resident;
  o->near_fp32 = P.near_fp32;
  o->deterministic = P.deterministic;
  o->colconv = P.cc.id >= 0 ? 1 : 0;
  o->near_assembly = P.near_assembly;
  o->pd_grid = P.pd_grid;
  o->pd_tol = P.near_assembly ? P.pd_tol : 0.0;
  o->near_seconds = P.near_seconds;
  o->assembly_seconds = P.assembly_seconds;
  o->bin_seconds = P.bin_seconds;
  o->symbol_seconds = P.symbol_seconds;
  o->row_pairs = (P.row_pairs && P.real_rows && P.rr.id >= 0 && P.cc.id >= 0 && P.rr.pairs) ? 1 : 0;
  return SBD_OK;
}

sbd_status sbd_plan_export(sbd_plan_t plan, int which, void* dst, size_t bytes) {
  if (!plan || !dst) return fail(SBD_EINVAL, "NULL argument");
  const Plan& P = *reinterpret_cast<Plan*>(plan);
  auto copy_dev = [&](const void* src, size_t need) {
    if (bytes < need) return fail(SBD_EINVAL, "destination too small");
    if (hipMemcpy(dst, src, need, hipMemcpyDeviceToHost) != hipSuccess) return fail(SBD_EHIP, "export copy");
    return SBD_OK;
  };
  auto copy_host = [&](const void* src, size_t need) {
    if (bytes < need) return fail(SBD_EINVAL, "destination too small");
    std::memcpy(dst, src, need);
    return SBD_OK;
  };
  switch (which) {
    case SBD_ARR_PERM: return copy_dev(P.perm, P.n * 4);
    case SBD_ARR_ROWPTR: return copy_dev(P.row_ptr, (P.n_tgt + 1) * 8);
    case SBD_ARR_TPERM: return copy_dev(P.tperm, P.n_tgt * 4);
    case SBD_ARR_COL: return copy_dev(P.col, P.nnz * 4);
    case SBD_ARR_VAL: {
      if (P.val) return copy_dev(P.val, P.nnz * 8);
      // near_fp32 plans keep D in FP32 only: widen on the host
      if (bytes < (size_t)P.nnz * 8) return fail(SBD_EINVAL, "destination too small");
      std::vector<float> v(P.nnz);
      if (hipMemcpy(v.data(), P.valf, P.nnz * 4, hipMemcpyDeviceToHost) != hipSuccess)
        return fail(SBD_EHIP, "export copy");
      double* d = (double*)dst;
      for (int64_t i = 0; i < P.nnz; ++i) d[i] = v[i];
      return SBD_OK;
    }
    case SBD_ARR_COEF: return copy_host(P.fit.coef.data(), P.fit.P * 8);
    case SBD_ARR_RADII: return copy_host(P.fit.radii.data(), P.fit.P * 8);
    case SBD_ARR_M: return copy_host(P.fit.M.data(), P.fit.P * 8);
    case SBD_ARR_KEYS:
    case SBD_ARR_TKEYS: {
      const int64_t cnt = which == SBD_ARR_KEYS ? P.n : P.n_tgt;
      const int32_t* src = which == SBD_ARR_KEYS ? P.skeys : P.tskeys;
      if (bytes < (size_t)cnt * 8) return fail(SBD_EINVAL, "destination too small");
      std::vector<int32_t> k(cnt);
      if (hipMemcpy(k.data(), src, cnt * 4, hipMemcpyDeviceToHost) != hipSuccess) return fail(SBD_EHIP, "export copy");
      int64_t* d = (int64_t*)dst;
      for (int64_t i = 0; i < cnt; ++i) d[i] = k[i];
      return SBD_OK;
    }
  }
  return fail(SBD_EINVAL, "unknown array");
}

void sbd_free(sbd_plan_t plan) {
  if (!plan) return;
  delete reinterpret_cast<Plan*>(plan);
}

sbd_status sbd_fft2(void* data, int64_t ny, int64_t nx, int dtype, int dir, void* stream) {
  if (!data || ny < 1 || nx < 1 || (dir != -1 && dir != 1)) return fail(SBD_EINVAL, "bad arguments");
  if (!is_smooth(ny) || !is_smooth(nx)) return fail(SBD_EINVAL, "sizes must be 7-smooth");
  if (dtype != SBD_C128 && dtype != SBD_C64) return fail(SBD_EINVAL, "complex dtype required");
  bool dbl = dtype == SBD_C128;
  hipStream_t st = (hipStream_t)stream;
  AxisPlan ax, ay;
  void* tmp = nullptr;
  size_t bytes = (size_t)nx * ny * (dbl ? 16 : 8);
  auto done = [&](sbd_status s) {
    free_axis_plan(ax);
    free_axis_plan(ay);
    if (tmp) (void)hipFree(tmp);
    return s;
  };
  if (build_axis_plan(ax, nx, dbl, max_lds(), 1) || build_axis_plan(ay, ny, dbl, max_lds(), 16))
    return done(fail(SBD_ENOMEM, "FFT plan"));
  if (hipMalloc(&tmp, bytes) != hipSuccess) return done(fail(SBD_ENOMEM, "FFT temporary"));
  int rc = 0;
  auto reorder = [&](int to_natural) {
    int r = dbl ? launch_reorder<double>(to_natural ? tmp : data, to_natural ? data : tmp, nx, ny, ax.store_L1,
                                         ax.store_L2, ay.store_L1, ay.store_L2, to_natural, st)
                : launch_reorder<float>(to_natural ? tmp : data, to_natural ? data : tmp, nx, ny, ax.store_L1,
                                        ax.store_L2, ay.store_L1, ay.store_L2, to_natural, st);
    return r;
  };
  if (dir < 0) {
    rc = dbl ? fft_rows<double>((double2*)data, ny, nx, 1, 0, ax, -1, INT64_MAX, INT64_MAX, st)
             : fft_rows<float>((float2*)data, ny, nx, 1, 0, ax, -1, INT64_MAX, INT64_MAX, st);
    if (!rc) rc = dbl ? fft_cols<double>((double2*)data, nx, nx, 1, 0, ay, -1, INT64_MAX, INT64_MAX, nullptr, 0, 16, st)
                      : fft_cols<float>((float2*)data, nx, nx, 1, 0, ay, -1, INT64_MAX, INT64_MAX, nullptr, 0, 16, st);
    // storage order -> natural order
    if (!rc && hipMemcpyAsync(tmp, data, bytes, hipMemcpyDeviceToDevice, st) != hipSuccess) rc = -5;
    if (!rc) rc = reorder(1);
  } else {
    // natural order -> storage order, then the inverse passes
    rc = reorder(0);
    if (!rc && hipMemcpyAsync(data, tmp, bytes, hipMemcpyDeviceToDevice, st) != hipSuccess) rc = -5;
    if (!rc) rc = dbl ? fft_cols<double>((double2*)data, nx, nx, 1, 0, ay, +1, INT64_MAX, INT64_MAX, nullptr, 0, 16, st)
                      : fft_cols<float>((float2*)data, nx, nx, 1, 0, ay, +1, INT64_MAX, INT64_MAX, nullptr, 0, 16, st);
    if (!rc) rc = dbl ? fft_rows<double>((double2*)data, ny, nx, 1, 0, ax, +1, INT64_MAX, INT64_MAX, st)
                      : fft_rows<float>((float2*)data, ny, nx, 1, 0, ax, +1, INT64_MAX, INT64_MAX, st);
  }
  hipError_t e = hipStreamSynchronize(st);
  if (rc || e != hipSuccess) return done(fail(SBD_EHIP, "fft kernels"));
  return done(SBD_OK);
}

}  // extern "C"
