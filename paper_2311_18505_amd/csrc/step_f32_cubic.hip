// FP32 (compensated) stepping kernels of the bow family with the cubic grid
// interpolant.
#include "step_kernel.h"

namespace sfd {
SFD_STEP_FAMILY(f32_cubic, float, true, true, true)
}  // namespace sfd
