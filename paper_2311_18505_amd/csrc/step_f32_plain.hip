// FP32 (compensated) stepping kernels without the bow family's code.
#include "step_kernel.h"

namespace sfd {
SFD_STEP_FAMILY(f32_plain, float, true, false, false)
}  // namespace sfd
