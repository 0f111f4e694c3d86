// Whole-column convolution pass for gfx950, specialised at compile time.
//
// A column of length L = R0 R1 R2 R3 lives in LDS (one column per 256-thread workgroup,
// two workgroups per CU).  The forward transform is a self-sorting Stockham sequence of
// radices (R0, R1, R2, R3) and the inverse one of (R3, R2, R1, R0): stage s with radix R
// and Ns = product of the earlier radices takes, for butterfly j, the inputs j + r L/R,
// multiplies input r by W_{Ns R}^{r (j mod Ns)}, performs an R-point DFT in registers and
// writes output r to (j div Ns) Ns R + (j mod Ns) + r Ns.  With every length, radix and
// stride a compile-time constant, LDS addresses fold into immediate offsets and no
// runtime index arithmetic remains beyond one quotient per butterfly.
//
// Three facts of the Toeplitz convolution shorten the work:
//  * the input column is zero beyond n_in <= L/2, so the first forward stage (R0 even)
//    reads its R0/2 lower inputs straight from global memory, and its butterflies fold
//    the zero upper half away;
//  * the last forward stage (R3, Ns = L/R3) writes frequency j + r L/R3 for butterfly j,
//    exactly the inputs of butterfly j of the first inverse stage (R3, Ns = 1): the two
//    stages and the symbol multiply run in registers with no LDS exchange between them;
//  * only rows e < n_out <= L/2 are kept, so the last inverse stage (R0, Ns = L/R0)
//    computes and stores its outputs r < R0/2 only.
// LDS holds one padding element after every R0 elements, which spreads the stride-R0
// writes of the first stage (and the strided writes of the others) over the banks.
#include <algorithm>
#include <cmath>
#include <vector>

#include "colconv.h"
#include "colconv_instances.h"

namespace sbd {

namespace cc {
#define SBD_CC_DECL(L, a, b, c, d, tag) int launch_##tag##_##L(const CcArgs&, int64_t, hipStream_t);
SBD_CC_F32R_A(SBD_CC_DECL)
SBD_CC_F32R_B(SBD_CC_DECL)
SBD_CC_F32C(SBD_CC_DECL)
SBD_CC_F64R(SBD_CC_DECL)
SBD_CC_F64C(SBD_CC_DECL)
#undef SBD_CC_DECL
}  // namespace cc

namespace {

using cc::CcArgs;

// exp(-2 pi i num / den) in FP64
inline void unit_root(int64_t num, int64_t den, double& c, double& s) {
  const double ang = -6.283185307179586476925286766559 * ((double)(num % den) / (double)den);
  c = std::cos(ang);
  s = std::sin(ang);
}

// twiddles of stage (R, Ns) at [k][r - 1] = W_{Ns R}^{dir r k}, dir = -1 forward, +1 inverse
void push_stage(std::vector<double2>& h, int R, int Ns, int dir) {
  for (int k = 0; k < Ns; ++k)
    for (int r = 1; r < R; ++r) {
      double c, s;
      unit_root((int64_t)r * k, (int64_t)Ns * R, c, s);
      h.push_back(make_double2(c, dir < 0 ? s : -s));
    }
}

// compiled instances: length, radices {R0, R1, R2, R3}, precision, complex symbol, launcher
struct CcInst {
  int L;
  int r[4];
  bool dbl, ch;
  int (*launch)(const CcArgs&, int64_t, hipStream_t);
};
const CcInst kInst[] = {
#define SBD_CC_F32R(L, a, b, c, d, tag) {L, {a, b, c, d}, false, false, cc::launch_##tag##_##L},
#define SBD_CC_F32X(L, a, b, c, d, tag) {L, {a, b, c, d}, false, true, cc::launch_##tag##_##L},
#define SBD_CC_F64X(L, a, b, c, d, tag) {L, {a, b, c, d}, true, false, cc::launch_##tag##_##L},
#define SBD_CC_F64Y(L, a, b, c, d, tag) {L, {a, b, c, d}, true, true, cc::launch_##tag##_##L},
    SBD_CC_F32R_A(SBD_CC_F32R) SBD_CC_F32R_B(SBD_CC_F32R) SBD_CC_F32C(SBD_CC_F32X) SBD_CC_F64R(SBD_CC_F64X)
    SBD_CC_F64C(SBD_CC_F64Y)
#undef SBD_CC_F32R
#undef SBD_CC_F32X
#undef SBD_CC_F64X
#undef SBD_CC_F64Y
};
constexpr int kNInst = (int)(sizeof(kInst) / sizeof(kInst[0]));

int inst_id(int64_t L, bool dbl, bool ch) {
  for (int i = 0; i < kNInst; ++i)
    if (kInst[i].dbl == dbl && kInst[i].ch == ch && kInst[i].L == L) return i;
  return -1;
}

template <typename T>
__global__ void k_store_symbol_cols(const double2* __restrict__ emb, int64_t Mx, int64_t My, int64_t ncols, int64_t e1x,
                                    int64_t e2x, int64_t e1y, int64_t e2y, double scale, int complex_out, void* out) {
  const int64_t ky = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t kx = blockIdx.y;
  const int64_t H = My / 2 + 1;
  if (ky >= H || kx >= ncols) return;
  const int64_t src = ((ky % e1y) * e2y + ky / e1y) * Mx + (kx % e1x) * e2x + kx / e1x;
  const double2 v = emb[src];
  const int64_t i = kx * H + ky;
  if (complex_out) reinterpret_cast<cplx<T>*>(out)[i] = mk<T>((T)(v.x * scale), (T)(v.y * scale));
  else reinterpret_cast<T*>(out)[i] = (T)(v.x * scale);
}

}  // namespace

bool colconv_available(int64_t L, bool is_double, bool complex_symbol) {
  return inst_id(L, is_double, complex_symbol) >= 0;
}

int64_t colconv_size(int64_t n, bool is_double, bool complex_symbol) {
  int64_t best = 0;
  for (int i = 0; i < kNInst; ++i)
    if (kInst[i].dbl == is_double && kInst[i].ch == complex_symbol && kInst[i].L >= n && (!best || kInst[i].L < best))
      best = kInst[i].L;
  return best;
}

int build_colconv_plan(ColConvPlan& cp, int64_t L, bool is_double, bool complex_symbol) {
  cp.id = inst_id(L, is_double, complex_symbol);
  cp.L = L;
  cp.is_double = is_double;
  cp.ch = complex_symbol;
  if (cp.id < 0) return -1;
  const int* r = kInst[cp.id].r;
  std::vector<double2> h;
  push_stage(h, r[1], r[0], -1);
  push_stage(h, r[2], r[0] * r[1], -1);
  push_stage(h, r[3], r[0] * r[1] * r[2], -1);
  push_stage(h, r[2], r[3], +1);
  push_stage(h, r[1], r[3] * r[2], +1);
  push_stage(h, r[0], r[3] * r[2] * r[1], +1);
  const size_t es = is_double ? 16 : 8;
  std::vector<unsigned char> bytes(h.size() * es);
  for (size_t i = 0; i < h.size(); ++i) {
    if (is_double) reinterpret_cast<double2*>(bytes.data())[i] = h[i];
    else reinterpret_cast<float2*>(bytes.data())[i] = make_float2((float)h[i].x, (float)h[i].y);
  }
  if (dev_malloc(&cp.tw, bytes.size()) != hipSuccess) { cp.tw = nullptr; return -2; }
  if (dev_upload(cp.tw, bytes.data(), bytes.size()) != hipSuccess) return -2;
  return 0;
}

void free_colconv_plan(ColConvPlan& cp) {
  dev_free(cp.tw);
  cp.tw = nullptr;
  cp.id = -1;
}

template <typename T>
int colconv(cplx<T>* data, int64_t ncols, int64_t pitch, int64_t nbatch, int64_t sbatch, const ColConvPlan& cp,
            int64_t n_in, int64_t n_out, const void* sym, int sym_complex, int64_t Mx, int ilv, hipStream_t st) {
  if (ncols > Mx || (ilv != 1 && ilv != 2)) return -1;
  if (ncols > pitch) return -1;  // (a row pair's 2 ncols elements fill at most its two rows)
  if (cp.id < 0 || cp.is_double != (sizeof(T) == 8) || cp.ch != (sym_complex != 0) || 2 * n_in > cp.L ||
      2 * n_out > cp.L || ncols < 1)
    return -1;
  if ((int64_t)cp.L * pitch * (int64_t)sizeof(cplx<T>) >= ((int64_t)1 << 40)) return -1;
  CcArgs a;
  a.data = data;
  a.pitch = pitch;
  a.ncols = ncols;
  a.sbatch = sbatch;
  a.n_in = (int)n_in;
  a.n_out = (int)n_out;
  a.tw = cp.tw;
  a.sym = sym;
  a.mx = Mx;
  a.ilv = ilv;
  int rc = kInst[cp.id].launch(a, nbatch, st);
  if (rc) return rc;
  // algorithmic bytes: the n_in input rows read, the n_out rows written, the half symbol
  const double e = sizeof(cplx<T>);
  mark_launch("fft_fused_mult", st,
              (double)nbatch * (double)ncols * (double)(n_in + n_out) * e +
                  (double)std::min<int64_t>(ncols, Mx / 2 + 1) * (double)(cp.L / 2 + 1) * (sym_complex ? e : e / 2));
  return 0;
}

template <typename T>
int store_symbol_cols(const double2* emb, int64_t Mx, int64_t My, int64_t ncols, int64_t e1x, int64_t e2x,
                      int64_t e1y, int64_t e2y, double scale, int complex_out, void* out, hipStream_t st) {
  const int64_t H = My / 2 + 1;
  dim3 grid((unsigned)ceil_div(H, 256), (unsigned)ncols);
  hipLaunchKernelGGL(k_store_symbol_cols<T>, grid, dim3(256), 0, st, emb, Mx, My, ncols, e1x, e2x, e1y, e2y, scale,
                     complex_out, out);
  return hipGetLastError() == hipSuccess ? 0 : -5;
}

template int colconv<float>(float2*, int64_t, int64_t, int64_t, int64_t, const ColConvPlan&, int64_t, int64_t,
                            const void*, int, int64_t, int, hipStream_t);
template int colconv<double>(double2*, int64_t, int64_t, int64_t, int64_t, const ColConvPlan&, int64_t, int64_t,
                             const void*, int, int64_t, int, hipStream_t);
template int store_symbol_cols<float>(const double2*, int64_t, int64_t, int64_t, int64_t, int64_t, int64_t, int64_t,
                                      double, int, void*, hipStream_t);
template int store_symbol_cols<double>(const double2*, int64_t, int64_t, int64_t, int64_t, int64_t, int64_t, int64_t,
                                       double, int, void*, hipStream_t);

}  // namespace sbd
