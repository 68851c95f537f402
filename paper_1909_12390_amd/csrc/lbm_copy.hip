// Streaming device-to-device copy: the measured HBM ceiling the step's kernels are
// compared with (every byte read once and written once, no reuse).  Each thread
// moves 16-byte vectors with non-temporal loads and stores (the lines are not kept
// in the caches), two vectors in flight per loop trip.  Measured on 2 GiB with
// 256-thread workgroups (GB/s, median of three): two in flight 5,155 / 5,432 /
// 5,141 at 8192 / 16384 / 32768 workgroups, one 5,006 / 5,247 / 5,193, four
// 5,090 / 5,101 / 5,077; cached loads or stores 4,200-4,900.
#include <hip/hip_runtime.h>

#include "lbm.h"
#include "lbm_internal.hpp"

namespace {

typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void k_stream_copy(const u32x4* __restrict__ src, u32x4* __restrict__ dst,
                                                     size_t n) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i + stride < n; i += 2 * stride) {
    const u32x4 a = __builtin_nontemporal_load(src + i);
    const u32x4 b = __builtin_nontemporal_load(src + i + stride);
    __builtin_nontemporal_store(a, dst + i);
    __builtin_nontemporal_store(b, dst + i + stride);
  }
  for (; i < n; i += stride) __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

}  // namespace

extern "C" lbm_status lbm_stream_copy(void* dst, const void* src, size_t bytes, int grid, void* stream) {
  if (!dst || !src || bytes % 16 != 0 || grid < 0)
    return lbm_fail(LBM_ERR_ARG, "lbm_stream_copy: null pointer, size not a multiple of 16 or negative grid");
  if (((uintptr_t)dst | (uintptr_t)src) % 16 != 0) return lbm_fail(LBM_ERR_ARG, "lbm_stream_copy: 16-byte alignment");
  if (bytes == 0) return LBM_OK;
  const size_t n = bytes / 16;
  const int blocks = grid > 0 ? grid : 256 * 8;
  hipLaunchKernelGGL(k_stream_copy, dim3(blocks), dim3(256), 0, (hipStream_t)stream, (const u32x4*)src, (u32x4*)dst,
                     n);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return lbm_fail(LBM_ERR_HIP, "stream copy launch: %s", hipGetErrorString(e));
  return LBM_OK;
}
