// Real-row transforms of the spread grid for gfx950, specialised at compile time.
//
// The real grid rows (length nx, zero-padded to M = 2 N) are transformed through one
// complex FFT of length N on z[j] = F[2j] + i F[2j+1] (the standard real-data split),
// with N = R0 R1 R2 R3 and every stride a compile-time constant, in the same Stockham
// stages as the column convolution.  The forward transform gathers its first stage's
// inputs straight from the tile subgrids (the upper half of z is zero padding, so stage 0
// takes only its R0/2 lower inputs); the inverse forms its first stage's inputs from
// X[k] and X[N - k] straight from the row and keeps only the outputs below nx/2 in its
// last stage.
#include <algorithm>
#include <cmath>
#include <vector>

#include "rows.h"
#include "rows_kernel.h"
#include "rows_instances.h"

namespace sbd {

namespace rr {
#define SBD_RR_DECL(N, a, b, c, d, tag)                                   \
  int launch_##tag##_fwd_##N(const RowArgs&, hipStream_t);               \
  int launch_##tag##_inv_##N(const RowArgs&, hipStream_t);
SBD_RR_F32(SBD_RR_DECL)
SBD_RR_F64(SBD_RR_DECL)
#undef SBD_RR_DECL
}  // namespace rr

namespace {

using rr::RowArgs;

inline void unit_root(int64_t num, int64_t den, double& c, double& s) {
  const double ang = -6.283185307179586476925286766559 * ((double)(num % den) / (double)den);
  c = std::cos(ang);
  s = std::sin(ang);
}

void push_stage(std::vector<double2>& h, int R, int Ns, int dir) {
  for (int k = 0; k < Ns; ++k)
    for (int r = 1; r < R; ++r) {
      double c, s;
      unit_root((int64_t)r * k, (int64_t)Ns * R, c, s);
      h.push_back(make_double2(c, dir < 0 ? s : -s));
    }
}

struct RrInst {
  int N;
  int r[4];
  bool dbl;
  bool pairs;                // has the two-rows-per-workgroup kernels
  int (*fwd)(const RowArgs&, hipStream_t);
  int (*inv)(const RowArgs&, hipStream_t);
};
const RrInst kInst[] = {
#define SBD_RR_E32(N, a, b, c, d, tag) \
  {N, {a, b, c, d}, false, rr::row_pairs_ok<float, a, b, c, d>(), rr::launch_##tag##_fwd_##N, rr::launch_##tag##_inv_##N},
#define SBD_RR_E64(N, a, b, c, d, tag) \
  {N, {a, b, c, d}, true, rr::row_pairs_ok<double, a, b, c, d>(), rr::launch_##tag##_fwd_##N, rr::launch_##tag##_inv_##N},
    SBD_RR_F32(SBD_RR_E32) SBD_RR_F64(SBD_RR_E64)
#undef SBD_RR_E32
#undef SBD_RR_E64
};
constexpr int kNInst = (int)(sizeof(kInst) / sizeof(kInst[0]));

void* upload(const std::vector<double2>& h, bool dbl) {
  const size_t es = dbl ? 16 : 8;
  std::vector<unsigned char> bytes(h.size() * es);
  for (size_t i = 0; i < h.size(); ++i) {
    if (dbl) reinterpret_cast<double2*>(bytes.data())[i] = h[i];
    else reinterpret_cast<float2*>(bytes.data())[i] = make_float2((float)h[i].x, (float)h[i].y);
  }
  void* p = nullptr;
  if (dev_malloc(&p, bytes.size()) != hipSuccess) return nullptr;
  if (dev_upload(p, bytes.data(), bytes.size()) != hipSuccess) {
    dev_free(p);
    return nullptr;
  }
  return p;
}

}  // namespace

int64_t rows_size(int64_t n, bool is_double) {
  int64_t best = 0;
  for (int i = 0; i < kNInst; ++i)
    if (kInst[i].dbl == is_double && kInst[i].N >= n && (!best || kInst[i].N < best)) best = kInst[i].N;
  return best;
}

int build_row_plan(RowPlan& rp, int64_t N, bool is_double) {
  rp.id = -1;
  for (int i = 0; i < kNInst; ++i)
    if (kInst[i].dbl == is_double && kInst[i].N == N) rp.id = i;
  rp.N = N;
  rp.is_double = is_double;
  if (rp.id < 0) return -1;
  rp.pairs = kInst[rp.id].pairs;
  const int* r = kInst[rp.id].r;
  std::vector<double2> h;
  push_stage(h, r[1], r[0], -1);
  push_stage(h, r[2], r[0] * r[1], -1);
  push_stage(h, r[3], r[0] * r[1] * r[2], -1);
  push_stage(h, r[2], r[3], +1);
  push_stage(h, r[1], r[3] * r[2], +1);
  push_stage(h, r[0], r[3] * r[2] * r[1], +1);
  std::vector<double2> m(N + 1);
  for (int64_t k = 0; k <= N; ++k) {
    double c, s;
    unit_root(k, 2 * N, c, s);
    m[k] = make_double2(c, s);
  }
  rp.tw = upload(h, is_double);
  rp.twM = upload(m, is_double);
  return (rp.tw && rp.twM) ? 0 : -2;
}

void free_row_plan(RowPlan& rp) {
  dev_free(rp.tw);
  dev_free(rp.twM);
  rp.tw = rp.twM = nullptr;
  rp.id = -1;
}

template <typename T, bool FWD>
int rows_cc(cplx<T>* grid, const RealRowArgs& a, const RowPlan& rp, hipStream_t st) {
  if (rp.id < 0 || rp.is_double != (sizeof(T) == 8) || a.nx > rp.N || a.M != 2 * rp.N) return -1;
  if (FWD && ((a.T & 1) || (a.SG & 1))) return -1;  // the forward gather reads cell pairs
  // row pairs: whole pairs of elements per (even) row start, and the two-rows-per-workgroup
  // inverse for this instance
  if (a.pair && ((a.gpitch & 1) || (a.sbatch & 1) || !rp.pairs)) return -1;
  RowArgs k;
  k.grid = grid;
  k.a = a;
  k.tw = rp.tw;
  k.twM = rp.twM;
  const int rc = FWD ? kInst[rp.id].fwd(k, st) : kInst[rp.id].inv(k, st);
  if (rc) return rc;
  const double elem = sizeof(cplx<T>);
  const double b = FWD ? (double)a.nbatch * ((double)a.ntiles * a.SG * a.SG * (elem / 2) + (double)a.ny * (rp.N + 1) * elem)
                       : (double)a.nbatch * (double)a.ny * ((rp.N + 1) * elem + (double)a.nx * elem / 2);
  mark_launch(FWD ? "fft_rows_r2c" : "fft_rows_c2r", st, b);
  return 0;
}

template <typename T>
int rows_r2c_cc(cplx<T>* grid, const RealRowArgs& a, const RowPlan& rp, hipStream_t st) {
  return rows_cc<T, true>(grid, a, rp, st);
}
template <typename T>
int rows_c2r_cc(cplx<T>* grid, const RealRowArgs& a, const RowPlan& rp, hipStream_t st) {
  return rows_cc<T, false>(grid, a, rp, st);
}
template int rows_r2c_cc<float>(float2*, const RealRowArgs&, const RowPlan&, hipStream_t);
template int rows_r2c_cc<double>(double2*, const RealRowArgs&, const RowPlan&, hipStream_t);
template int rows_c2r_cc<float>(float2*, const RealRowArgs&, const RowPlan&, hipStream_t);
template int rows_c2r_cc<double>(double2*, const RealRowArgs&, const RowPlan&, hipStream_t);

}  // namespace sbd
