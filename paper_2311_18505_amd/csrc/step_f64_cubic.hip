// FP64 stepping kernels of the bow family with the cubic grid interpolant.
#include "step_kernel.h"

namespace sfd {
SFD_STEP_FAMILY(f64_cubic, double, false, true, true)
}  // namespace sfd
