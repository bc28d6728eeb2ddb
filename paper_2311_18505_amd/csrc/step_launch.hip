// Launch dispatch of the stepping kernels and the auxiliary kernels of
// libstringfdtd (rewind, gather, bulk upload, counters, delay).
#include <hip/hip_runtime.h>

#include "sfd_types.h"

namespace sfd {

// one pair of host entry points per instantiation family (step_*.hip)
#define SFD_DECLARE_FAMILY(NAME)                                                               \
  hipError_t launch_step_##NAME(int kernel, const LaunchArgs &a, int blocks, hipStream_t st); \
  int blocks_step_##NAME(int kernel);
SFD_DECLARE_FAMILY(f32_plain)
SFD_DECLARE_FAMILY(f32_bow)
SFD_DECLARE_FAMILY(f32_cubic)
SFD_DECLARE_FAMILY(f64_plain)
SFD_DECLARE_FAMILY(f64_bow)
SFD_DECLARE_FAMILY(f64_cubic)
#undef SFD_DECLARE_FAMILY

__global__ void zero_counters(int32_t *c, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) c[i] = 0;
}

// Restores slots first..first+count-1 to their state right after excitation:
// one block per slot copies the saved state block and the saved status.
template <typename T>
__global__ void rewind_kernel(const Desc *desc, Status *status, const Status *status0, int first, int count) {
  const int s = first + (int)blockIdx.x;
  if ((int)blockIdx.x >= count) return;
  const Desc &D = desc[s];
  if (!D.st0) return;
  T *dst = (T *)D.st;
  const T *src = (const T *)D.st0;
  for (int i = (int)threadIdx.x; i < D.st_elems; i += (int)blockDim.x) dst[i] = src[i];
  if (threadIdx.x == 0) status[s] = status0[s];
}

// Row i of dst receives samples offs[i] .. offs[i]+count-1 of slot slots[i]'s
// output; samples the slot has not produced (at or past its samples_done, or
// past n_samples) are written as zero.  The slot's samples_done and flags go
// to row_done[i] and row_flags[i].  One block per row.
template <typename T>
__global__ void gather_kernel(const Desc *desc, const Status *status, const int32_t *slots, const int64_t *offs,
                              int n, int64_t count, T *dst, int64_t *row_done, int32_t *row_flags) {
  const int i = (int)blockIdx.x;
  if (i >= n) return;
  const int s = slots[i];
  const Desc &D = desc[s];
  const int64_t done = status[s].samples_done;
  const int64_t avail = (done < D.n_samples ? done : D.n_samples) - offs[i];
  const int64_t c = count < avail ? count : (avail > 0 ? avail : 0);
  const T *src = (const T *)D.out + offs[i];
  for (int64_t t = threadIdx.x; t < count; t += blockDim.x) dst[(int64_t)i * count + t] = t < c ? src[t] : T(0);
  if (threadIdx.x == 0) {
    row_done[i] = done;
    row_flags[i] = status[s].flags;
  }
}

hipError_t launch_gather(int precision, const Desc *desc, const Status *status, const int32_t *slots,
                         const int64_t *offs, int n, int64_t count, void *dst, int64_t *row_done, int32_t *row_flags,
                         hipStream_t st) {
  if (n <= 0) return hipSuccess;
  if (precision == 1)
    hipLaunchKernelGGL(gather_kernel<float>, dim3(n), dim3(256), 0, st, desc, status, slots, offs, n, count,
                       (float *)dst, row_done, row_flags);
  else
    hipLaunchKernelGGL(gather_kernel<double>, dim3(n), dim3(256), 0, st, desc, status, slots, offs, n, count,
                       (double *)dst, row_done, row_flags);
  return hipGetLastError();
}

// Bulk upload: segment i copies bytes[i] bytes (a multiple of 4) from
// src + src_off[i] to dst[i], one block per segment.
__global__ void scatter_kernel(const uint32_t *src, const UploadSeg *segs, int n) {
  const int i = (int)blockIdx.x;
  if (i >= n) return;
  const UploadSeg g = segs[i];
  const uint32_t *from = src + g.src_off / 4;
  uint32_t *to = (uint32_t *)g.dst;
  for (uint64_t w = threadIdx.x; w < g.bytes / 4; w += blockDim.x) to[w] = from[w];
}

hipError_t launch_scatter(const void *src, const UploadSeg *segs, int n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(scatter_kernel, dim3(n), dim3(256), 0, st, (const uint32_t *)src, segs, n);
  return hipGetLastError();
}

hipError_t launch_rewind(int precision, const Desc *desc, Status *status, const Status *status0, int first, int count,
                         hipStream_t st) {
  if (count <= 0) return hipSuccess;
  if (precision == 1)
    hipLaunchKernelGGL(rewind_kernel<float>, dim3(count), dim3(256), 0, st, desc, status, status0, first, count);
  else
    hipLaunchKernelGGL(rewind_kernel<double>, dim3(count), dim3(256), 0, st, desc, status, status0, first, count);
  return hipGetLastError();
}

// kernel: 0 the merged classes 0..4, 1..3 the classes 5..7 (kernel_of_class);
// variant: kVarPlain, kVarBow or kVarCubic; precision 1 is FP32 with
// compensation, else FP64
hipError_t launch_kernel(int precision, int kernel, int variant, const LaunchArgs &a, int blocks, hipStream_t st) {
  if (precision == 1) {
    switch (variant) {
      case kVarPlain: return launch_step_f32_plain(kernel, a, blocks, st);
      case kVarBow: return launch_step_f32_bow(kernel, a, blocks, st);
      default: return launch_step_f32_cubic(kernel, a, blocks, st);
    }
  }
  switch (variant) {
    case kVarPlain: return launch_step_f64_plain(kernel, a, blocks, st);
    case kVarBow: return launch_step_f64_bow(kernel, a, blocks, st);
    default: return launch_step_f64_cubic(kernel, a, blocks, st);
  }
}

// Holds its stream for `ticks` of the constant-rate wall clock and exits
// (bounded by time, independent of any other kernel).  Placed before the
// merged launch so that the two large-class launches, which need whole SIMDs
// (512 registers per wavefront), are dispatched before the merged launch's
// persistent wavefronts fill every CU.
__global__ void delay_kernel(uint64_t ticks) {
  const uint64_t t0 = wall_clock64();
  // the iteration cap bounds the wait (~20 ms) even if the clock stood still
  for (int i = 0; i < 100000 && wall_clock64() - t0 < ticks; ++i) __builtin_amdgcn_s_sleep(8);
}

hipError_t launch_delay(uint64_t ticks, hipStream_t st) {
  hipLaunchKernelGGL(delay_kernel, dim3(1), dim3(64), 0, st, ticks);
  return hipGetLastError();
}

hipError_t launch_zero(int32_t *c, int n, hipStream_t st) {
  hipLaunchKernelGGL(zero_counters, dim3((n + 255) / 256), dim3(256), 0, st, c, n);
  return hipGetLastError();
}

int max_blocks_per_cu(int precision, int kernel, int variant) {
  if (precision == 1) {
    switch (variant) {
      case kVarPlain: return blocks_step_f32_plain(kernel);
      case kVarBow: return blocks_step_f32_bow(kernel);
      default: return blocks_step_f32_cubic(kernel);
    }
  }
  switch (variant) {
    case kVarPlain: return blocks_step_f64_plain(kernel);
    case kVarBow: return blocks_step_f64_bow(kernel);
    default: return blocks_step_f64_cubic(kernel);
  }
}

}  // namespace sfd
