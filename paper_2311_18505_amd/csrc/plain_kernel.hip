// Plain FP64 per-string method (eq. (7) as printed, banded LU): comparator path.
#include <hip/hip_runtime.h>

#include "sfd_types.h"

namespace sfd {

hipError_t launch_plain(const Desc *, Status *, int, int64_t, int, double, hipStream_t) {
  return hipErrorNotSupported;
}

}  // namespace sfd
