// Instances of the compiled whole-column convolution (split over several sources so the
// build compiles them in parallel).
#include "colconv_instances.h"
#include "colconv_kernel.h"

namespace sbd {
namespace cc {
#define SBD_CC_DEF(L, a, b, c, d, tag) \
  int launch_##tag##_##L(const CcArgs& x, int64_t nb, hipStream_t st) { return launch_inst<float, false, a, b, c, d>(x, nb, st); }
SBD_CC_F32R_A(SBD_CC_DEF)
#undef SBD_CC_DEF
}  // namespace cc
}  // namespace sbd
