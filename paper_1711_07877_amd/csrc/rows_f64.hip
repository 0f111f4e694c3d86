// Instances of the compiled real-row transforms (double).
#include "rows_instances.h"
#include "rows_kernel.h"

namespace sbd {
namespace rr {
#define SBD_RR_DEF(N, a, b, c, d, tag)                                                                              \
  int launch_##tag##_fwd_##N(const RowArgs& k, hipStream_t st) { return launch_row<double, true, a, b, c, d>(k, st); } \
  int launch_##tag##_inv_##N(const RowArgs& k, hipStream_t st) { return launch_row<double, false, a, b, c, d>(k, st); }
SBD_RR_F64(SBD_RR_DEF)
#undef SBD_RR_DEF
}  // namespace rr
}  // namespace sbd
