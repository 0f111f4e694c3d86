// Mixed-radix Stockham FFT passes held in LDS (gfx950, wave64).
//
// Each stage of radix R takes, for butterfly j of a length-L sequence with
// Ns = product of the previous radices, the inputs x[j + r L/R] (r < R),
// multiplies input r by W_{Ns R}^{r (j mod Ns)}, performs an R-point DFT and
// writes output r to position (j div Ns) Ns R + (j mod Ns) + r Ns (the
// self-sorting Stockham formulation).  All loads of a stage complete before a
// barrier, then all stores, so one LDS buffer suffices.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "dft.h"
#include "fft.h"
#include "gridrow.h"

namespace sbd {

namespace {

using dft::Dft;

// Exact quotient n / d for 0 <= n < 2^22 from a float reciprocal plus one
// correction step (the float estimate is within one of the true quotient).
__device__ __forceinline__ int qdiv(int n, int d, float inv) {
  int q = (int)((float)n * inv);
  int r = n - q * d;
  q += (r >= d) ? 1 : 0;
  q -= (r < 0) ? 1 : 0;
  return q;
}

// LDS layout: element e of sequence s lives at ((e + e / 16) * nseq + s); the pad
// element every 16 breaks the power-of-two strides of early Stockham stages.  The
// number of interleaved sequences nseq is a power of two, passed as lg = log2(nseq).
__device__ __forceinline__ int lds_index(int e, int lg, int s) { return ((e + (e >> 4)) << lg) + s; }
__host__ __device__ inline size_t lds_elems(int L, int nseq) { return (size_t)(L + (L >> 4) + 1) * (size_t)nseq; }

// One Stockham stage over nseq interleaved sequences.
// Twiddles W_L^m come from two small tables in LDS: W_L^m = coarse[m >> 7] * fine[m & 127],
// fine[i] = W_L^i (i < 128) and coarse[c] = W_L^(128 c).
constexpr int kTwFine = 128;
__host__ __device__ inline int tw_coarse(int L) { return (L + kTwFine - 1) / kTwFine; }
__host__ __device__ inline size_t tw_entries(int L) { return (size_t)kTwFine + (size_t)tw_coarse(L); }

template <typename T>
__device__ __forceinline__ cplx<T> twiddle(const cplx<T>* tw, int m) {
  return cmul<T>(tw[kTwFine + (m >> 7)], tw[m & (kTwFine - 1)]);
}

// LINR: every read stride L/R is a multiple of the pad period 16, so the padded index
// of leg r is lds_index(j) + r (L/R + L/(16 R)): one add per element.  Only compiled
// into whole kernels whose every stage qualifies (a per-stage choice inside one kernel
// makes the register allocation spill).
template <typename T, int R, int NB, bool TWLDS, bool LINR = false>
__device__ __forceinline__ void stage(cplx<T>* buf, int LR, int lgseq, int Ns, float inv_Ns, int tstep,
                                      const cplx<T>* __restrict__ tw, int dir) {
  // LR = L / R butterflies per sequence; tstep = L / (Ns R) (two-level table index step)
  const int nbf = LR << lgseq;
  const int smask = (1 << lgseq) - 1;
  cplx<T> v[NB][R];
  int dst[NB], sq[NB];
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    int t = threadIdx.x + i * blockDim.x;
    dst[i] = -1;
    sq[i] = 0;
    if (t < nbf) {
      const int j = t >> lgseq;
      const int s = t & smask;
      const int g = qdiv(j, Ns, inv_Ns);
      const int k = j - g * Ns;
      if constexpr (LINR) {
        const int base = lds_index(j, lgseq, s);
        const int step = (LR + (LR >> 4)) << lgseq;
#pragma unroll
        for (int r = 0; r < R; ++r) v[i][r] = buf[base + r * step];
      } else {
        int e = j;
#pragma unroll
        for (int r = 0; r < R; ++r) {
          v[i][r] = buf[lds_index(e, lgseq, s)];
          e += LR;
        }
      }
      if (Ns > 1) {
        const int kt = k * tstep;
#pragma unroll
        for (int r = 1; r < R; ++r) {
          // global per-stage table: W_{Ns R}^{r k} at [k][r - 1], so the lanes of a wave
          // (consecutive k) read consecutive entries
          cplx<T> w = TWLDS ? twiddle<T>(tw, r * kt) : tw[k * (R - 1) + (r - 1)];
          if (dir > 0) w.y = -w.y;
          v[i][r] = cmul<T>(v[i][r], w);
        }
      }
      Dft<T, R>::run(v[i], dir);
      dst[i] = j + (j - k) * (R - 1);  // = g Ns R + k
      sq[i] = s;
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    if (dst[i] >= 0) {
      int e = dst[i];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        buf[lds_index(e, lgseq, sq[i])] = v[i][r];
        e += Ns;
      }
    }
  }
  __syncthreads();
}

// tw: two-level table in LDS (TWLDS) or the per-stage tables in global memory
// (stage s holds W_{Ns R}^{r k} for k < Ns, r = 1..R-1, stages back to back).
// COMP: radix 12 is compiled in: FP32 row kernels, FP32 pass kernels with at most
// kCompositeMaxEpt elements per thread, and FP64 pass kernels with linear reads (see
// stage), which have the register headroom for it; other FP64 kernels, wider FP32
// pass kernels, and radix 6 anywhere, spill.
constexpr int kCompositeMaxEpt = 18;
template <typename T>
__host__ __device__ constexpr bool comp_compiled(int ept, bool linr) {
  return sizeof(T) == 4 ? ept <= kCompositeMaxEpt : linr;
}
template <typename T, int EPT, bool TWLDS = true, bool COMP = false, bool LINR = false>
__device__ void lds_fft(cplx<T>* buf, int L, int lgseq, const Radices& rad, const cplx<T>* tw, int dir) {
  int Ns = 1;
  int cur = L;  // L / Ns
  int64_t off = 0;
  for (int s = 0; s < rad.n; ++s) {
    const int R = rad.r[s];
    const float inv_Ns = 1.0f / (float)Ns;
    const cplx<T>* t = TWLDS ? tw : tw + off;
    switch (R) {
      case 8: stage<T, 8, (EPT + 7) / 8, TWLDS, LINR>(buf, L / 8, lgseq, Ns, inv_Ns, cur / 8, t, dir); break;
      case 4: stage<T, 4, (EPT + 3) / 4, TWLDS, LINR>(buf, L / 4, lgseq, Ns, inv_Ns, cur / 4, t, dir); break;
      case 2: stage<T, 2, (EPT + 1) / 2, TWLDS, LINR>(buf, L / 2, lgseq, Ns, inv_Ns, cur / 2, t, dir); break;
      case 3: stage<T, 3, (EPT + 2) / 3, TWLDS, LINR>(buf, L / 3, lgseq, Ns, inv_Ns, cur / 3, t, dir); break;
      case 5: stage<T, 5, (EPT + 4) / 5, TWLDS, LINR>(buf, L / 5, lgseq, Ns, inv_Ns, cur / 5, t, dir); break;
      case 7: stage<T, 7, (EPT + 6) / 7, TWLDS, LINR>(buf, L / 7, lgseq, Ns, inv_Ns, cur / 7, t, dir); break;
      // composite radices: FP32 plans only (see factor)
      case 9:
        if constexpr (sizeof(T) == 4) stage<T, 9, (EPT + 8) / 9, TWLDS, LINR>(buf, L / 9, lgseq, Ns, inv_Ns, cur / 9, t, dir);
        break;
      case 12:
        if constexpr (COMP) stage<T, 12, (EPT + 11) / 12, TWLDS, LINR>(buf, L / 12, lgseq, Ns, inv_Ns, cur / 12, t, dir);
        break;
      default: break;
    }
    off += (int64_t)Ns * (R - 1);
    Ns *= R;
    cur /= R;
  }
}

template <typename T>
struct KArgs {
  cplx<T>* data;
  PassDesc d;
  const cplx<T>* twL;
  const cplx<T>* twFull;   // non-null: per-stage twiddle tables read from global memory (strided passes)
  const cplx<T>* twM;
  int dir;
  // fused multiply (+ inverse) mode
  const void* mult;
  int mult_complex;
  int64_t sO3;
};

template <typename T, int EPT, bool FUSED, bool LINR>
__global__ void __launch_bounds__(1024) k_fft_pass(KArgs<T> a) {
  extern __shared__ unsigned char smem_raw[];
  cplx<T>* buf = reinterpret_cast<cplx<T>*>(smem_raw);
  const PassDesc& d = a.d;
  const int64_t nib = (d.nInner + d.Bi - 1) / d.Bi;
  int64_t bx = blockIdx.x;
  if (d.xcd_remap) {
    // blocks are dispatched round-robin over the 8 XCDs: give each XCD a
    // contiguous range of logical blocks so neighbouring columns share its L2
    const int64_t nb = (int64_t)gridDim.x;
    const int64_t q = nb >> 3, rem = nb & 7, x = bx & 7;
    bx = x * q + (x < rem ? x : rem) + (bx >> 3);
  }
  const int64_t ib = bx % nib;
  const int64_t o1 = bx / nib;
  const int64_t o2 = blockIdx.y;
  const int64_t o3 = blockIdx.z;
  const int Bi = d.Bi;
  const int lgBi = d.lgBi;
  const int L = d.L;
  const int64_t inner0 = ib * Bi;
  const int bvalid = (int)((d.nInner - inner0) < Bi ? (d.nInner - inner0) : Bi);
  cplx<T>* g = a.data + o3 * a.sO3 + o2 * d.sO2 + o1 * d.sO1 + inner0;
  const int total = L * Bi;
  const int64_t lgbase = o1 * d.lgO + inner0 * d.lgI;
  cplx<T>* twl = buf + lds_elems(L, Bi);
  const bool tw_in_lds = a.twFull == nullptr;
  if (tw_in_lds)
    for (int i = threadIdx.x; i < (int)tw_entries(L); i += blockDim.x) twl[i] = a.twL[i];
  for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
    int e = idx >> lgBi;
    int b = idx & (Bi - 1);
    cplx<T> v = mk<T>(T(0), T(0));
    int64_t lg = e * d.lgE + lgbase + b * d.lgI;
    if (b < bvalid && lg < d.n_in) {
      v = g[e * d.sE + b];
      if (d.tw_mode == 2) {  // inverse four-step: pre-twiddle W_M^{+e q}
        int64_t q = (inner0 + b) * d.twI + o1 * d.twO;
        cplx<T> w = a.twM[e * q];
        w.y = -w.y;
        v = cmul<T>(v, w);
      }
    }
    buf[lds_index(e, lgBi, b)] = v;
  }
  __syncthreads();
  // radix 12 only where the register budget leaves room for it (see factor)
  constexpr bool kComp = comp_compiled<T>(EPT, LINR);
  if (tw_in_lds) lds_fft<T, EPT, true, kComp, LINR>(buf, L, lgBi, d.rad, twl, a.dir);
  else lds_fft<T, EPT, false, kComp, LINR>(buf, L, lgBi, d.rad, a.twFull, a.dir);
  if (FUSED) {
    const int64_t mbase = o1 * d.sO1 + inner0;
    for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
      int e = idx >> lgBi;
      int b = idx & (Bi - 1);
      if (b < bvalid) {
        int64_t off = mbase + e * d.sE + b;
        int li = lds_index(e, lgBi, b);
        if (a.mult_complex) {
          cplx<T> m = reinterpret_cast<const cplx<T>*>(a.mult)[off];
          buf[li] = cmul<T>(buf[li], m);
        } else {
          T m = reinterpret_cast<const T*>(a.mult)[off];
          buf[li] = cscale<T>(buf[li], m);
        }
      }
    }
    __syncthreads();
    if (tw_in_lds) lds_fft<T, EPT, true, kComp, LINR>(buf, L, lgBi, d.rad, twl, +1);
    else lds_fft<T, EPT, false, kComp, LINR>(buf, L, lgBi, d.rad, a.twFull, +1);
  }
  for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
    int e = idx >> lgBi;
    int b = idx & (Bi - 1);
    int64_t lg = e * d.lgE + lgbase + b * d.lgI;
    if (b < bvalid && lg < d.n_out) {
      cplx<T> v = buf[lds_index(e, lgBi, b)];
      if (d.tw_mode == 1) {  // forward four-step: post-twiddle W_M^{-e q}
        int64_t q = (inner0 + b) * d.twI + o1 * d.twO;
        v = cmul<T>(v, a.twM[e * q]);
      }
      g[e * d.sE + b] = v;
    }
  }
}

// Stockham stages.  Every stage costs an LDS round trip, two barriers and its index
// and twiddle work, so fewer, larger butterflies are cheaper.  FP64 plans take
// powers of two in 8s, then 3, 5, 7 (larger FP64 butterflies exceed the register
// budget of 1024-thread workgroups); FP32 plans pair threes into radix 9.  With
// composite radix 12 joins (FP64: without 9), and the sequence
// with the fewest stages is taken, ties broken by an estimate of the arithmetic per
// element (largest radices first).
double radix_work(int R) {
  // approximate real flops per element of one stage: butterfly + input twiddles
  double bf = R == 2 ? 2 : R == 3 ? 7 : R == 4 ? 4 : R == 5 ? 10 : R == 7 ? 13 : R == 8 ? 7.5 : R == 9 ? 16 : 12.7;
  return bf + 6.0 * (R - 1) / R;
}

void search_radices(int64_t x, int maxR, int depth, int* cur, int* best, int& best_n, double& best_c, double c,
                    bool is_double) {
  static const int kSet[] = {12, 9, 8, 7, 5, 4, 3, 2};
  if (x == 1) {
    if (depth < best_n || (depth == best_n && c < best_c - 1e-9)) {
      best_n = depth;
      best_c = c;
      for (int i = 0; i < depth; ++i) best[i] = cur[i];
    }
    return;
  }
  if (depth + 1 >= kMaxStages || depth + 1 > best_n) return;
  for (int R : kSet) {
    if (R > maxR || x % R || (is_double && R == 9)) continue;
    cur[depth] = R;
    search_radices(x / R, R, depth + 1, cur, best, best_n, best_c, c + radix_work(R), is_double);
  }
}

void factor(int64_t L, Radices& r, bool is_double, bool composite = false) {
  r.n = 0;
  auto push = [&](int R) { if (r.n < kMaxStages) r.r[r.n++] = R; };
  static int mode = -1;  // SBD_FFT_FACTOR=greedy: no radix 12
  if (mode < 0) {
    const char* env = getenv("SBD_FFT_FACTOR");
    mode = (env && strcmp(env, "greedy") == 0) ? 0 : 1;
  }
  if (composite && mode == 1) {
    int cur[kMaxStages], best[kMaxStages];
    int best_n = kMaxStages;
    double best_c = 1e300;
    search_radices(L, 12, 0, cur, best, best_n, best_c, 0.0, is_double);
    if (best_n < kMaxStages) {
      for (int i = 0; i < best_n; ++i) push(best[i]);
      return;
    }
  }
  int64_t x = L;
  int a2 = 0, a3 = 0, a5 = 0, a7 = 0;
  while (x % 2 == 0) { ++a2; x /= 2; }
  while (x % 3 == 0) { ++a3; x /= 3; }
  while (x % 5 == 0) { ++a5; x /= 5; }
  while (x % 7 == 0) { ++a7; x /= 7; }
  for (; a2 >= 3; a2 -= 3) push(8);
  if (a2 == 2) push(4);
  if (a2 == 1) push(2);
  if (!is_double)
    for (; a3 >= 2; a3 -= 2) push(9);
  for (; a3 >= 1; --a3) push(3);
  for (; a5 >= 1; --a5) push(5);
  for (; a7 >= 1; --a7) push(7);
}

// exp(-2 pi i num / den) in FP64 (the angle's rounding, about 1e-16 relative, is far
// below every transform's tolerance)
inline void unit_root(int64_t num, int64_t den, double& c, double& s) {
  const double ang = -6.283185307179586476925286766559 * ((double)(num % den) / (double)den);
  c = std::cos(ang);
  s = std::sin(ang);
}

// Per-stage twiddles for the radix sequence rad of a length-L transform: for
// stage s (Ns = product of the earlier radices, radix R) the entries
// W_{Ns R}^{r k} at [k][r - 1], k < Ns, r = 1..R-1; stages back to back.
template <typename T>
void* make_stage_table(const Radices& rad) {
  std::vector<cplx<T>> h;
  int64_t Ns = 1;
  for (int s = 0; s < rad.n; ++s) {
    const int R = rad.r[s];
    for (int64_t k = 0; k < Ns; ++k)
      for (int r = 1; r < R; ++r) {
        double c, sn;
        unit_root(r * k, Ns * R, c, sn);
        h.push_back(mk<T>((T)c, (T)sn));
      }
    Ns *= R;
  }
  void* p = nullptr;
  if (h.empty()) h.push_back(mk<T>(T(1), T(0)));
  if (dev_malloc(&p, h.size() * sizeof(cplx<T>)) != hipSuccess) return nullptr;
  if (dev_upload(p, h.data(), h.size() * sizeof(cplx<T>)) != hipSuccess) return nullptr;
  return p;
}

template <typename T>
void* make_full_table(int64_t L) {
  std::vector<cplx<T>> h(L);
  for (int64_t m = 0; m < L; ++m) {
    double c, sn;
    unit_root(m, L, c, sn);
    h[m] = mk<T>((T)c, (T)sn);
  }
  void* p = nullptr;
  if (dev_malloc(&p, L * sizeof(cplx<T>)) != hipSuccess) return nullptr;
  if (dev_upload(p, h.data(), L * sizeof(cplx<T>)) != hipSuccess) return nullptr;
  return p;
}

// Two-level table for W_L^m: [fine (128 entries) | coarse (ceil(L/128) entries)].
template <typename T>
void* make_table(int64_t L) {
  const int nc = tw_coarse((int)L);
  std::vector<cplx<T>> h(kTwFine + nc);
  for (int i = 0; i < kTwFine; ++i) {
    double c, sn;
    unit_root(i, L, c, sn);
    h[i] = mk<T>((T)c, (T)sn);
  }
  for (int c = 0; c < nc; ++c) {
    double cc, sn;
    unit_root((int64_t)c * kTwFine, L, cc, sn);
    h[kTwFine + c] = mk<T>((T)cc, (T)sn);
  }
  void* p = nullptr;
  if (dev_malloc(&p, h.size() * sizeof(cplx<T>)) != hipSuccess) return nullptr;
  if (dev_upload(p, h.data(), h.size() * sizeof(cplx<T>)) != hipSuccess) return nullptr;
  return p;
}

int g_ept_target = 0;

void choose_threads(PassDesc& d, size_t elem) {
  d.lgBi = 0;
  while ((1 << d.lgBi) < d.Bi) ++d.lgBi;  // Bi is a power of two
  if (g_ept_target == 0) {
    const char* env = getenv("SBD_FFT_EPT");
    g_ept_target = env ? std::max(4, std::min(32, atoi(env))) : 32;
  }
  int64_t tot = (int64_t)d.L * d.Bi;
  const int cap = elem > 8 ? std::min(g_ept_target, 12) : std::min(g_ept_target, 24);
  int nthr = 64;
  while (nthr < 1024 && ceil_div(tot, nthr) > cap) nthr *= 2;
  int64_t ept = ceil_div(tot, nthr);
  d.nthreads = nthr;
  // smallest instantiated register budget covering the actual elements per thread
  d.ept = ept <= 4 ? 4 : ept <= 8 ? 8 : ept <= 12 ? 12 : ept <= 16 ? 16 : ept <= 18 ? 18 : ept <= 24 ? 24 : 32;
  // wider register budgets spill (FP32 above 24, FP64 above 12 elements per thread):
  // such a pass is refused rather than run slowly
  if (ept > (elem > 8 ? 12 : 24)) d.ept = 0;
  d.lds_bytes = (lds_elems(d.L, d.Bi) + tw_entries(d.L)) * elem;
}

// Algorithmic bytes of one pass: every element of the transformed region that
// may be non-zero is read once, every stored element written once, plus the
// multiplier in the fused pass (twiddle tables are not counted).
double pass_bytes(const PassDesc& d, int64_t axis_len, size_t elem, int64_t nO3, const void* mult, int mult_complex) {
  double total = (double)d.L * (double)d.nInner * (double)d.nO1 * (double)d.nO2 * (double)nO3;
  double fin = (double)std::min<int64_t>(d.n_in, axis_len) / (double)axis_len;
  double fout = (double)std::min<int64_t>(d.n_out, axis_len) / (double)axis_len;
  double b = total * (double)elem * (fin + fout);
  if (mult) b += total / (double)nO3 * (double)(mult_complex ? elem : elem / 2);
  return b;
}

// Every stage's read stride L/R is a multiple of the LDS pad period (stage, LINR).
bool linear_reads(int64_t L, const Radices& rad) {
  if (rad.n == 0) return false;
  for (int s = 0; s < rad.n; ++s)
    if ((L / rad.r[s]) % 16) return false;
  return true;
}

// Every radix of rad has a butterfly compiled into the kernel instance (type, EPT,
// composite flag): a missing one would leave its stage out, so such a pass is refused.
bool radices_supported(const Radices& rad, bool is_double, bool comp) {
  for (int s = 0; s < rad.n; ++s) {
    const int R = rad.r[s];
    if (R == 2 || R == 3 || R == 4 || R == 5 || R == 7 || R == 8) continue;
    if (R == 9 && !is_double) continue;
    if (R == 12 && comp) continue;
    return false;
  }
  return true;
}

template <typename T>
int launch(cplx<T>* data, const PassDesc& d, const void* twL, const void* twM, int dir,
           const void* mult, int mult_complex, int64_t nO3, int64_t sO3, hipStream_t st, int64_t axis_len,
           const void* twFull = nullptr) {
  KArgs<T> a;
  a.data = data;
  a.d = d;
  a.twL = (const cplx<T>*)twL;
  a.twFull = (const cplx<T>*)twFull;
  a.twM = (const cplx<T>*)twM;
  a.dir = dir;
  a.mult = mult;
  a.mult_complex = mult_complex;
  a.sO3 = sO3;
  int64_t nib = ceil_div(d.nInner, d.Bi);
  dim3 grid((unsigned)(nib * d.nO1), (unsigned)d.nO2, (unsigned)nO3);
  dim3 block(d.nthreads);
  bool fused = mult != nullptr;
  const bool lin = linear_reads(d.L, d.rad);
  if (d.ept == 0 || !radices_supported(d.rad, sizeof(T) == 8, comp_compiled<T>(d.ept, lin))) return -1;
#define SBD_L(E)                                                                                     \
  do {                                                                                               \
    auto kfn = lin ? (fused ? (void (*)(KArgs<T>))k_fft_pass<T, E, true, true>                       \
                            : (void (*)(KArgs<T>))k_fft_pass<T, E, false, true>)                     \
                   : (fused ? (void (*)(KArgs<T>))k_fft_pass<T, E, true, false>                      \
                            : (void (*)(KArgs<T>))k_fft_pass<T, E, false, false>);                   \
    if (d.lds_bytes > 65536)                                                                         \
      (void)hipFuncSetAttribute((const void*)kfn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)d.lds_bytes); \
    hipLaunchKernelGGL(kfn, grid, block, d.lds_bytes, st, a);                                        \
  } while (0)
  if (d.ept == 0) return -1;
  switch (d.ept) {
    case 4: SBD_L(4); break;
    case 8: SBD_L(8); break;
    case 12: SBD_L(12); break;
    case 16: SBD_L(16); break;
    case 18: SBD_L(18); break;
    case 24: SBD_L(24); break;
    default: SBD_L(32); break;
  }
#undef SBD_L
  if (hipGetLastError() != hipSuccess) return -5;
  mark_launch(fused ? "fft_fused_mult" : (d.tw_mode ? "fft_fourstep_A" : (d.sE == 1 ? "fft_contig" : "fft_strided")), st,
              pass_bytes(d, axis_len, sizeof(cplx<T>), nO3, mult, mult_complex));
  return 0;
}

template <typename T>
struct RealKArgs {
  cplx<T>* grid;
  RealRowArgs a;
  int64_t N;
  Radices rad;
  const cplx<T>* twN;
  const cplx<T>* twM;
  const cplx<T>* twS;   // non-null: per-stage tables in global memory instead of the LDS table
};

template <typename T, int EPT>
__global__ void __launch_bounds__(1024) k_rows_r2c(RealKArgs<T> k) {
  extern __shared__ unsigned char smem_raw[];
  cplx<T>* buf = reinterpret_cast<cplx<T>*>(smem_raw);
  const RealRowArgs& a = k.a;
  const int64_t Y = blockIdx.x;
  const int64_t r = blockIdx.y;
  const int64_t N = k.N;
  cplx<T>* twl = buf + lds_elems((int)N, 1);
  if (!k.twS)
    for (int i = threadIdx.x; i < (int)tw_entries((int)N); i += blockDim.x) twl[i] = k.twN[i];
  const cplx<T>* sub2 = reinterpret_cast<const cplx<T>*>(a.sub);
  // tile rows covering grid row Y: ty = Y >> log2T and ty - 1 (if the halo reaches)
  const int tyhi = (int)(Y >> a.log2T);
  int64_t row0 = -1, row1 = -1;
  int ly0 = 0, ly1 = 0;
  if (tyhi < a.nty) { ly0 = (int)(Y - ((int64_t)tyhi << a.log2T)); if (ly0 < a.SG) row0 = r * a.ntiles + (int64_t)tyhi * a.ntx; }
  if (tyhi >= 1 && tyhi - 1 < a.nty) {
    ly1 = (int)(Y - ((int64_t)(tyhi - 1) << a.log2T));
    if (ly1 < a.SG) row1 = r * a.ntiles + (int64_t)(tyhi - 1) * a.ntx;
  }
  for (int j = threadIdx.x; j < N; j += blockDim.x) buf[lds_index(j, 0, 0)] = gather_pair<T>(sub2, a, 2 * j, ly0, ly1, row0, row1);
  __syncthreads();
  if (k.twS) lds_fft<T, EPT, false, sizeof(T) == 4>(buf, (int)N, 0, k.rad, k.twS, -1);
  else lds_fft<T, EPT, true, sizeof(T) == 4>(buf, (int)N, 0, k.rad, twl, -1);
  cplx<T>* out = k.grid + r * a.sbatch + Y * a.gpitch;
  for (int64_t q = threadIdx.x; q <= N; q += blockDim.x) {
    cplx<T> zk = buf[lds_index(q == N ? 0 : (int)q, 0, 0)];
    cplx<T> zc = buf[lds_index(q == 0 ? 0 : (int)(N - q), 0, 0)];
    zc.y = -zc.y;  // conj(Z[N - k])
    cplx<T> E = mk<T>(T(0.5) * (zk.x + zc.x), T(0.5) * (zk.y + zc.y));
    // O = (Z[k] - conj(Z[N-k])) / (2i)
    cplx<T> D = mk<T>(T(0.5) * (zk.x - zc.x), T(0.5) * (zk.y - zc.y));
    cplx<T> O = mk<T>(D.y, -D.x);
    out[q] = cadd<T>(E, cmul<T>(k.twM[q], O));
  }
}

template <typename T, int EPT>
__global__ void __launch_bounds__(1024) k_rows_c2r(RealKArgs<T> k) {
  extern __shared__ unsigned char smem_raw[];
  cplx<T>* buf = reinterpret_cast<cplx<T>*>(smem_raw);
  const RealRowArgs& a = k.a;
  const int64_t Y = blockIdx.x;
  const int64_t r = blockIdx.y;
  const int64_t N = k.N;
  cplx<T>* row = k.grid + r * a.sbatch + Y * a.gpitch;
  cplx<T>* twl = buf + lds_elems((int)N, 1);
  if (!k.twS)
    for (int i = threadIdx.x; i < (int)tw_entries((int)N); i += blockDim.x) twl[i] = k.twN[i];
  for (int64_t q = threadIdx.x; q < N; q += blockDim.x) {
    cplx<T> xk = row[q];
    cplx<T> xc = row[N - q];
    xc.y = -xc.y;  // conj(X[N - k])
    cplx<T> A = cadd<T>(xk, xc);
    cplx<T> w = k.twM[q];
    w.y = -w.y;  // W_M^{-k}
    cplx<T> B = cmul<T>(csub<T>(xk, xc), w);
    buf[lds_index((int)q, 0, 0)] = mk<T>(A.x - B.y, A.y + B.x);  // A + i B
  }
  __syncthreads();
  if (k.twS) lds_fft<T, EPT, false, sizeof(T) == 4>(buf, (int)N, 0, k.rad, k.twS, +1);
  else lds_fft<T, EPT, true, sizeof(T) == 4>(buf, (int)N, 0, k.rad, twl, +1);
  T* outr = reinterpret_cast<T*>(row);
  for (int64_t j = threadIdx.x; 2 * j < a.nx; j += blockDim.x) {
    cplx<T> z = buf[lds_index((int)j, 0, 0)];
    outr[2 * j] = z.x;
    if (2 * j + 1 < a.nx) outr[2 * j + 1] = z.y;
  }
}

template <typename T, bool FWD>
int launch_real_rows(cplx<T>* grid, const RealRowArgs& a, const RealRowPlan& rp, hipStream_t st) {
  RealKArgs<T> k;
  k.grid = grid;
  k.a = a;
  k.N = rp.N;
  k.rad = rp.r;
  k.twN = (const cplx<T>*)rp.twN;
  k.twM = (const cplx<T>*)rp.twM;
  k.twS = (const cplx<T>*)rp.twS;
  PassDesc d;
  d.L = (int)rp.N;
  d.Bi = 1;
  choose_threads(d, sizeof(cplx<T>));
  if (d.ept == 0 || !radices_supported(rp.r, sizeof(T) == 8, sizeof(T) == 4)) return -1;
  if (FWD && ((a.T & 1) || (a.SG & 1))) return -1;  // the forward gather reads cell pairs
  dim3 grid_dim((unsigned)a.ny, (unsigned)a.nbatch);
#define SBD_RL(E)                                                                                         \
  do {                                                                                                    \
    auto kfn = FWD ? (void (*)(RealKArgs<T>))k_rows_r2c<T, E> : (void (*)(RealKArgs<T>))k_rows_c2r<T, E>; \
    if (d.lds_bytes > 65536)                                                                              \
      (void)hipFuncSetAttribute((const void*)kfn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)d.lds_bytes); \
    hipLaunchKernelGGL(kfn, grid_dim, dim3(d.nthreads), d.lds_bytes, st, k);                              \
  } while (0)
  switch (d.ept) {
    case 4: SBD_RL(4); break;
    case 8: SBD_RL(8); break;
    case 12: SBD_RL(12); break;
    case 16: SBD_RL(16); break;
    case 18: SBD_RL(18); break;
    case 24: SBD_RL(24); break;
    default: SBD_RL(32); break;
  }
#undef SBD_RL
  if (hipGetLastError() != hipSuccess) return -5;
  const double elem = sizeof(cplx<T>);
  double b;
  if (FWD) {
    b = (double)a.nbatch * ((double)a.ntiles * a.SG * a.SG * (elem / 2) + (double)a.ny * (rp.N + 1) * elem);
  } else {
    b = (double)a.nbatch * (double)a.ny * ((rp.N + 1) * elem + (double)a.nx * elem / 2);
  }
  mark_launch(FWD ? "fft_rows_r2c" : "fft_rows_c2r", st, b);
  return 0;
}

}  // namespace

int build_real_row_plan(RealRowPlan& rp, int64_t M, bool is_double, size_t max_lds) {
  if (M % 2) return -1;
  rp.N = M / 2;
  rp.is_double = is_double;
  size_t elem = is_double ? 16 : 8;
  if ((lds_elems((int)rp.N, 1) + tw_entries((int)rp.N)) * elem > max_lds || !is_smooth(rp.N)) return -1;
  factor(rp.N, rp.r, is_double, !is_double);
  if (is_double) {
    rp.twN = make_table<double>(rp.N);
    rp.twS = make_stage_table<double>(rp.r);
    std::vector<double2> h(rp.N + 1);
    for (int64_t k = 0; k <= rp.N; ++k) {
      double c, sn;
      unit_root(k, M, c, sn);
      h[k] = make_double2(c, sn);
    }
    if (dev_malloc(&rp.twM, h.size() * sizeof(double2)) != hipSuccess) return -2;
    if (dev_upload(rp.twM, h.data(), h.size() * sizeof(double2)) != hipSuccess) return -2;
  } else {
    rp.twN = make_table<float>(rp.N);
    rp.twS = make_stage_table<float>(rp.r);
    std::vector<float2> h(rp.N + 1);
    for (int64_t k = 0; k <= rp.N; ++k) {
      double c, sn;
      unit_root(k, M, c, sn);
      h[k] = make_float2((float)c, (float)sn);
    }
    if (dev_malloc(&rp.twM, h.size() * sizeof(float2)) != hipSuccess) return -2;
    if (dev_upload(rp.twM, h.data(), h.size() * sizeof(float2)) != hipSuccess) return -2;
  }
  return (rp.twN && rp.twS) ? 0 : -2;
}

void free_real_row_plan(RealRowPlan& rp) {
  dev_free(rp.twN);
  dev_free(rp.twS);
  dev_free(rp.twM);
  rp.twN = rp.twM = rp.twS = nullptr;
}

template <typename T>
int rows_r2c(cplx<T>* grid, const RealRowArgs& a, const RealRowPlan& rp, hipStream_t st) {
  return launch_real_rows<T, true>(grid, a, rp, st);
}
template <typename T>
int rows_c2r(cplx<T>* grid, const RealRowArgs& a, const RealRowPlan& rp, hipStream_t st) {
  return launch_real_rows<T, false>(grid, a, rp, st);
}
template int rows_r2c<float>(float2*, const RealRowArgs&, const RealRowPlan&, hipStream_t);
template int rows_r2c<double>(double2*, const RealRowArgs&, const RealRowPlan&, hipStream_t);
template int rows_c2r<float>(float2*, const RealRowArgs&, const RealRowPlan&, hipStream_t);
template int rows_c2r<double>(double2*, const RealRowArgs&, const RealRowPlan&, hipStream_t);

bool is_smooth(int64_t n) {
  if (n <= 0) return false;
  for (int p : {2, 3, 5, 7})
    while (n % p == 0) n /= p;
  return n == 1;
}

int64_t best_fft_size(int64_t n, int64_t multiple_of, bool is_double) {
  // smooth size in [n, 1.08 n] minimising size x (weighted radix stages + 2): the LDS
  // kernels pay mostly per stage (one LDS round trip and two barriers each), and the
  // odd-radix butterflies (5, 7) cost more than the power-of-two and radix-3 ones
  int64_t best = next_smooth(n, multiple_of);
  double bestc = 1e300;
  for (int64_t m = best; m <= std::max<int64_t>(best, (int64_t)(1.08 * (double)n)); ++m) {
    if (!is_smooth(m) || m % multiple_of) continue;
    Radices r;
    factor(m, r, is_double);
    double st = 0.0;
    for (int i = 0; i < r.n; ++i) st += r.r[i] == 7 ? 2.0 : r.r[i] == 5 ? 1.5 : r.r[i] == 9 ? 1.3 : 1.0;
    double c = (double)m * (st + 2.0);
    if (c < bestc) { bestc = c; best = m; }
  }
  return best;
}

int64_t next_smooth(int64_t n, int64_t multiple_of) {
  int64_t m = n < 1 ? 1 : n;
  while (!(is_smooth(m) && m % multiple_of == 0)) ++m;
  return m;
}

int build_axis_plan(AxisPlan& ap, int64_t M, bool is_double, size_t max_lds, int bi_strided) {
  ap.M = M;
  ap.is_double = is_double;
  size_t elem = is_double ? 16 : 8;
  auto need = [&](int64_t L, int bi) { return (lds_elems((int)L, bi) + tw_entries((int)L)) * elem; };
  ap.single_bi = 0;
  if (bi_strided > 1 && need(M, bi_strided) > max_lds) {
    // strided (column) axis: hold whole columns in LDS when one fits
    const char* env = getenv("SBD_COLS_SINGLE");
    int allow = env ? atoi(env) : 1;
    // (one column per block already beats the three-pass four-step split in FP64)
    int bi = 0;  // largest power of two (<= bi_strided) whose columns fit
    if (need(M, 1) <= max_lds) {
      bi = 1;
      while (bi * 2 <= bi_strided && need(M, bi * 2) <= max_lds) bi *= 2;
    }
    const char* cap = getenv("SBD_COLS_BI");  // optional cap on the columns per block
    if (cap && atoi(cap) >= 1)
      while (bi > atoi(cap)) bi /= 2;
    if (allow && bi >= 1) ap.single_bi = bi;
  }
  // single pass if the strided batch fits in LDS
  ap.four_step = need(M, bi_strided) > max_lds;
  if (!ap.four_step) {
    ap.L1 = (int)M;
    ap.L2 = 1;
  } else {
    // split M = L1 * L2 with L1 <= L2, both as close to sqrt(M) as possible
    int best = 0;
    for (int64_t l1 = 2; l1 * l1 <= M; ++l1)
      if (M % l1 == 0 && is_smooth(l1) && is_smooth(M / l1)) best = (int)l1;
    if (best == 0) return -1;
    ap.L1 = best;
    ap.L2 = (int)(M / best);
    if (need(ap.L2, bi_strided) > max_lds) return -1;
  }
  factor(ap.L1, ap.r1, is_double);
  factor(ap.L2, ap.r2, is_double);
  ap.store_L1 = (ap.single_bi > 0 || !ap.four_step) ? (int)M : ap.L1;
  ap.store_L2 = (ap.single_bi > 0 || !ap.four_step) ? 1 : ap.L2;
  if (ap.single_bi > 0) {
    // the whole-column pass may use radix 12 when it runs at most kCompositeMaxEpt
    // elements per thread (the launch picks the same width from the same descriptor)
    PassDesc probe;
    probe.L = (int)M;
    probe.Bi = ap.single_bi;
    choose_threads(probe, elem);
    if (!is_double) {
      factor(M, ap.rs, false, probe.ept > 0 && probe.ept <= kCompositeMaxEpt);
    } else {
      // FP64: radix 12 only in kernels with linear reads, so only when every stage qualifies
      factor(M, ap.rs, true, true);
      if (!linear_reads(M, ap.rs)) factor(M, ap.rs, true, false);
    }
    ap.twS = is_double ? make_table<double>(M) : make_table<float>(M);
    ap.twSfull = is_double ? make_stage_table<double>(ap.rs) : make_stage_table<float>(ap.rs);
    if (!ap.twS || !ap.twSfull) return -2;
  }
  if (is_double) {
    ap.tw1 = make_table<double>(ap.L1);
    ap.tw2 = ap.four_step ? make_table<double>(ap.L2) : nullptr;
    ap.twM = ap.four_step ? make_full_table<double>(M) : nullptr;
  } else {
    ap.tw1 = make_table<float>(ap.L1);
    ap.tw2 = ap.four_step ? make_table<float>(ap.L2) : nullptr;
    ap.twM = ap.four_step ? make_full_table<float>(M) : nullptr;
  }
  if (!ap.tw1 || (ap.four_step && (!ap.tw2 || !ap.twM))) return -2;
  return 0;
}

void free_axis_plan(AxisPlan& ap) {
  dev_free(ap.tw1);
  dev_free(ap.tw2);
  dev_free(ap.twM);
  dev_free(ap.twS);
  dev_free(ap.twSfull);
  ap.tw1 = ap.tw2 = ap.twM = ap.twS = ap.twSfull = nullptr;
}

template <typename T>
int fft_rows(cplx<T>* data, int64_t nrows, int64_t pitch, int64_t nbatch, int64_t sbatch,
             const AxisPlan& ap, int dir, int64_t n_in, int64_t n_out, hipStream_t st) {
  const size_t elem = sizeof(cplx<T>);
  if (!ap.four_step) {
    PassDesc d;
    d.L = ap.L1;
    d.rad = ap.r1;
    d.sE = 1;
    d.Bi = 1;
    d.nInner = 1;
    d.sO1 = pitch;
    d.nO1 = nrows;
    d.lgE = 1;
    d.n_in = n_in;
    d.n_out = n_out;
    choose_threads(d, elem);
    return launch<T>(data, d, ap.tw1, nullptr, dir, nullptr, 0, nbatch, sbatch, st, ap.M);
  }
  const int L1 = ap.L1, L2 = ap.L2;
  // pass A: length-L1 FFTs over j1 (stride L2), inner j2 contiguous, outer row
  PassDesc A;
  A.L = L1;
  A.rad = ap.r1;
  A.sE = L2;
  A.Bi = 16;
  while (A.Bi > 1 && (lds_elems(L1, A.Bi) + tw_entries(L1)) * elem > 65536) A.Bi /= 2;
  A.nInner = L2;
  A.sO1 = pitch;
  A.nO1 = nrows;
  A.lgE = L2;
  A.lgI = 1;
  A.twI = 1;
  A.M = ap.M;
  choose_threads(A, elem);
  // pass B: length-L2 FFTs over contiguous runs, outer k1 (stride L2) and row
  PassDesc B;
  B.L = L2;
  B.rad = ap.r2;
  B.sE = 1;
  B.Bi = 1;
  B.nInner = 1;
  B.sO1 = L2;
  B.nO1 = L1;
  B.sO2 = pitch;
  B.nO2 = nrows;
  choose_threads(B, elem);
  int rc;
  if (dir < 0) {
    A.n_in = n_in;
    A.tw_mode = 1;
    rc = launch<T>(data, A, ap.tw1, ap.twM, dir, nullptr, 0, nbatch, sbatch, st, ap.M);
    if (rc) return rc;
    return launch<T>(data, B, ap.tw2, nullptr, dir, nullptr, 0, nbatch, sbatch, st, ap.M);
  }
  rc = launch<T>(data, B, ap.tw2, nullptr, dir, nullptr, 0, nbatch, sbatch, st, ap.M);
  if (rc) return rc;
  A.tw_mode = 2;
  A.n_out = n_out;
  return launch<T>(data, A, ap.tw1, ap.twM, dir, nullptr, 0, nbatch, sbatch, st, ap.M);
}

template <typename T>
int fft_cols(cplx<T>* data, int64_t ncols, int64_t pitch, int64_t nbatch, int64_t sbatch,
             const AxisPlan& ap, int dir, int64_t n_in, int64_t n_out,
             const void* mult, int mult_complex, int Bi, hipStream_t st) {
  const size_t elem = sizeof(cplx<T>);
  if (ap.single_bi > 0 && ap.four_step) {
    // whole columns in LDS (a few per block, strided rows), XCD-aware block order
    PassDesc d;
    d.L = (int)ap.M;
    d.rad = ap.rs;
    d.sE = pitch;
    d.Bi = ap.single_bi;
    d.nInner = ncols;
    d.lgE = 1;
    d.n_in = n_in;
    d.n_out = (mult || dir > 0) ? n_out : INT64_MAX;
    d.xcd_remap = 1;
    choose_threads(d, elem);
    // twiddles: FP32 from the per-stage tables in global memory, FP64 from the two-level
    // LDS table (measured at 8640: FP32 525 against 545 us, FP64 981 against 1004 us);
    // SBD_COLS_TWLDS = 0 / 1 forces either
    static int tw_forced = -2;
    if (tw_forced == -2) {
      const char* env = getenv("SBD_COLS_TWLDS");
      tw_forced = env ? atoi(env) : -1;
    }
    const bool tw_lds = tw_forced >= 0 ? tw_forced != 0 : sizeof(T) == 8;
    return launch<T>(data, d, ap.twS, nullptr, mult ? -1 : dir, mult, mult_complex, nbatch, sbatch, st, ap.M,
                     tw_lds ? nullptr : ap.twSfull);
  }
  if (!ap.four_step) {
    PassDesc d;
    d.L = ap.L1;
    d.rad = ap.r1;
    d.sE = pitch;
    d.Bi = Bi;
    d.nInner = ncols;
    d.lgE = 1;
    d.n_in = n_in;
    d.n_out = (mult || dir > 0) ? n_out : INT64_MAX;
    choose_threads(d, elem);
    return launch<T>(data, d, ap.tw1, nullptr, mult ? -1 : dir, mult, mult_complex, nbatch, sbatch, st, ap.M);
  }
  const int L1 = ap.L1, L2 = ap.L2;
  PassDesc A;  // over j1: stride L2*pitch; outer j2 (stride pitch); inner columns
  A.L = L1;
  A.rad = ap.r1;
  A.sE = (int64_t)L2 * pitch;
  A.Bi = Bi;
  A.nInner = ncols;
  A.sO1 = pitch;
  A.nO1 = L2;
  A.lgE = L2;
  A.lgO = 1;
  A.twO = 1;
  A.M = ap.M;
  choose_threads(A, elem);
  PassDesc B;  // over j2: stride pitch; outer k1 (stride L2*pitch); inner columns
  B.L = L2;
  B.rad = ap.r2;
  B.sE = pitch;
  B.Bi = Bi;
  B.nInner = ncols;
  B.sO1 = (int64_t)L2 * pitch;
  B.nO1 = L1;
  choose_threads(B, elem);
  int rc;
  if (dir < 0 || mult) {
    A.n_in = n_in;
    A.tw_mode = 1;
    rc = launch<T>(data, A, ap.tw1, ap.twM, -1, nullptr, 0, nbatch, sbatch, st, ap.M);
    if (rc) return rc;
    rc = launch<T>(data, B, ap.tw2, nullptr, -1, mult, mult_complex, nbatch, sbatch, st, ap.M);
    if (rc || !mult) return rc;
  } else {
    rc = launch<T>(data, B, ap.tw2, nullptr, +1, nullptr, 0, nbatch, sbatch, st, ap.M);
    if (rc) return rc;
  }
  A.n_in = INT64_MAX;
  A.tw_mode = 2;
  A.n_out = n_out;
  return launch<T>(data, A, ap.tw1, ap.twM, +1, nullptr, 0, nbatch, sbatch, st, ap.M);
}

template int fft_rows<float>(float2*, int64_t, int64_t, int64_t, int64_t, const AxisPlan&, int, int64_t, int64_t, hipStream_t);
template int fft_rows<double>(double2*, int64_t, int64_t, int64_t, int64_t, const AxisPlan&, int, int64_t, int64_t, hipStream_t);
template int fft_cols<float>(float2*, int64_t, int64_t, int64_t, int64_t, const AxisPlan&, int, int64_t, int64_t, const void*, int, int, hipStream_t);
template int fft_cols<double>(double2*, int64_t, int64_t, int64_t, int64_t, const AxisPlan&, int, int64_t, int64_t, const void*, int, int, hipStream_t);

}  // namespace sbd
