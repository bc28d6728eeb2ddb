// Fixed device scratch of libstringfdtd for the entry points that allocate
// nothing (string_batch_gather_output_noalloc).
//
// The array lives in the library's code object: every GPU the library runs
// on holds its own copy, at its own address, from the first use until the
// process ends.  Host code never passes the array's name to a kernel (on the
// host it is only a stand-in for the symbol); it asks the runtime for the
// device address once per device and passes that.  Every call on one GPU
// shares the array: calls that overlap on one GPU (two batches on different
// streams at once) race on it.
#include <hip/hip_runtime.h>

#include <mutex>

#include "sfd_types.h"

namespace sfd {

static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void *g_scratch_ptr[kMaxDevices] = {};
}  // namespace

// Device address of `scratch` on `device` (the current device when called
// from the set-up of a batch), looked up once per device.
hipError_t static_scratch_ptr(int device, void **ptr) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_ptr[device]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_ptr[device] = p;
  }
  *ptr = g_scratch_ptr[device];
  return hipSuccess;
}

}  // namespace sfd
