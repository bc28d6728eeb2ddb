// FP64 stepping kernels without the bow family's code.
#include "step_kernel.h"

namespace sfd {
SFD_STEP_FAMILY(f64_plain, double, false, false, false)
}  // namespace sfd
