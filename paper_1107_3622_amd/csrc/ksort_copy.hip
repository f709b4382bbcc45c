// Streaming copy used as the bandwidth ceiling of a level pass.
//
// A level pass reads every live key once and writes it once; a plain device
// copy of the same bytes is the most a pass could reach on this GPU.  This
// kernel is that copy, written like the pass itself: a persistent grid of
// at most occupancy x compute units workgroups, 16-byte loads and stores
// per lane, four in flight per lane before the first store, and a
// workgroup-strided walk over 64 KiB chunks so each workgroup streams whole
// contiguous pieces.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>

#include "ksort.h"
#include "ksort_engine.h"

namespace ksort {

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));  // one 16-byte access

constexpr int kCopyBlock = 256;
constexpr int kCopyUnroll = 4;                                   // 16-byte accesses in flight per lane
constexpr int64_t kCopyChunk = (int64_t)kCopyBlock * kCopyUnroll * 16;  // bytes per workgroup step

__global__ __launch_bounds__(kCopyBlock) void stream_copy_kernel(u32x4* __restrict__ dst, const u32x4* __restrict__ src,
                                                                 int64_t n16) {
  const int64_t per = kCopyChunk / 16;
  for (int64_t base = (int64_t)blockIdx.x * per; base < n16; base += (int64_t)gridDim.x * per) {
    u32x4 v[kCopyUnroll];
    if (base + per <= n16) {
#pragma unroll
      for (int u = 0; u < kCopyUnroll; ++u) v[u] = src[base + u * kCopyBlock + threadIdx.x];
#pragma unroll
      for (int u = 0; u < kCopyUnroll; ++u) dst[base + u * kCopyBlock + threadIdx.x] = v[u];
    } else {
#pragma unroll
      for (int u = 0; u < kCopyUnroll; ++u) {
        const int64_t j = base + u * kCopyBlock + threadIdx.x;
        if (j < n16) dst[j] = src[j];
      }
    }
  }
}

__global__ void tail_copy_kernel(unsigned char* dst, const unsigned char* src, int64_t n) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j < n) dst[j] = src[j];
}

}  // namespace ksort

using namespace ksort;

extern "C" int ksort_stream_copy(void* d_dst, const void* d_src, size_t bytes, int grid, void* stream) {
  if (bytes == 0) return KSORT_OK;
  if (!d_dst || !d_src) return fail(KSORT_EINVAL, "null pointer");
  if (((uintptr_t)d_dst | (uintptr_t)d_src) % 16 != 0) return fail(KSORT_EINVAL, "buffers must be 16-byte aligned");
  int dev = 0;
  KSORT_HIP(hipGetDevice(&dev));
  if (grid <= 0) {
    int occ = 0, cus = 0;
    KSORT_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, (const void*)stream_copy_kernel, kCopyBlock, 0));
    KSORT_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    grid = std::max(1, occ * cus);
  }
  const int64_t n16 = (int64_t)(bytes / 16);
  const int64_t chunks = (n16 * 16 + kCopyChunk - 1) / kCopyChunk;
  grid = (int)std::max<int64_t>(1, std::min<int64_t>(grid, chunks));
  hipStream_t st = (hipStream_t)stream;
  if (n16 > 0) hipLaunchKernelGGL(stream_copy_kernel, dim3(grid), dim3(kCopyBlock), 0, st, (u32x4*)d_dst, (const u32x4*)d_src, n16);
  const int64_t rest = (int64_t)(bytes % 16);
  if (rest)
    hipLaunchKernelGGL(tail_copy_kernel, dim3(1), dim3(64), 0, st, (unsigned char*)d_dst + n16 * 16,
                       (const unsigned char*)d_src + n16 * 16, rest);
  KSORT_HIP(hipGetLastError());
  return KSORT_OK;
}
