// Instances of the compiled real-row transforms (float).
#include "rows_instances.h"
#include "rows_kernel.h"

namespace sbd {
namespace rr {
#define SBD_RR_DEF(N, a, b, c, d, tag)                                                                              \
  int launch_##tag##_fwd_##N(const RowArgs& k, hipStream_t st) { return launch_row<float, true, a, b, c, d>(k, st); } \
  int launch_##tag##_inv_##N(const RowArgs& k, hipStream_t st) { return launch_row<float, false, a, b, c, d>(k, st); }
SBD_RR_F32(SBD_RR_DEF)
#undef SBD_RR_DEF
}  // namespace rr
}  // namespace sbd
