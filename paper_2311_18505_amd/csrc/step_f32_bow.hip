// FP32 (compensated) stepping kernels of the bow family (bowed strings,
// clamped ends, the zeta channel, cubic hammers).
#include "step_kernel.h"

namespace sfd {
SFD_STEP_FAMILY(f32_bow, float, true, true, false)
}  // namespace sfd
