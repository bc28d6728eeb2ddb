// FP64 stepping kernels of the bow family.
#include "step_kernel.h"

namespace sfd {
SFD_STEP_FAMILY(f64_bow, double, false, true, false)
}  // namespace sfd
