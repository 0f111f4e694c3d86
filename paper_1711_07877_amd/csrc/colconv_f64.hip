// Instances of the compiled whole-column convolution (split over several sources so the
// build compiles them in parallel).
#include "colconv_instances.h"
#include "colconv_kernel.h"

namespace sbd {
namespace cc {
#define SBD_CC_DEFR(L, a, b, c, d, tag) \
  int launch_##tag##_##L(const CcArgs& x, int64_t nb, hipStream_t st) { return launch_inst<double, false, a, b, c, d>(x, nb, st); }
#define SBD_CC_DEFC(L, a, b, c, d, tag) \
  int launch_##tag##_##L(const CcArgs& x, int64_t nb, hipStream_t st) { return launch_inst<double, true, a, b, c, d>(x, nb, st); }
SBD_CC_F64R(SBD_CC_DEFR)
SBD_CC_F64C(SBD_CC_DEFC)
#undef SBD_CC_DEFR
#undef SBD_CC_DEFC
}  // namespace cc
}  // namespace sbd
