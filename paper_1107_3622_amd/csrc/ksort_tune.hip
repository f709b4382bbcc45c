// Autotuner: times every compiled kernel variant (threads per workgroup,
// keys per thread in a partition tile, LDS-finish cutoff) on a seeded
// U[0,1) input of the requested size and key type, and makes the fastest the
// default for inputs of about that size (the same power-of-two bucket, or
// the nearest tuned bucket at most two powers of two away).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "ksort.h"
#include "ksort_engine.h"

namespace ksort {

// Timing input: SplitMix64 (Steele, Lea, Flood, OOPSLA 2014) outputs mapped
// to U[0,1): 53 bits for double, 24 bits for float.
template <typename T>
__global__ void fill_uniform(T* out, int64_t n, uint64_t seed) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
    uint64_t z = seed + (uint64_t)(t + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    if (sizeof(T) == 8)
      out[t] = (T)((double)(z >> 11) * 0x1p-53);
    else
      out[t] = (T)((double)(z >> 40) * 0x1p-24);
  }
}

static std::mutex g_tuned_mu;
static std::map<std::pair<int, int>, ksort_tuning> g_tuned;  // (dtype, log2 bucket) -> variant

static int bucket_of(int64_t n) { return n <= 1 ? 0 : (int)std::floor(std::log2((double)n)); }

bool tuned_for(int dtype, int64_t n, ksort_tuning* out) {
  std::lock_guard<std::mutex> lk(g_tuned_mu);
  const int b = bucket_of(n);
  for (int d = 0; d <= 2; ++d) {
    for (int sgn : {1, -1}) {
      auto it = g_tuned.find({dtype, b + sgn * d});
      if (it != g_tuned.end()) {
        *out = it->second;
        return true;
      }
      if (d == 0) break;
    }
  }
  return false;
}

static int time_variant(int dtype, const ksort_tuning& tn, void* src, void* work, int64_t n, size_t kb,
                        hipStream_t st, int reps, double* best_ms) {
  hipEvent_t e0, e1;
  KSORT_HIP(hipEventCreate(&e0));
  KSORT_HIP(hipEventCreate(&e1));
  double best = 1e30;
  int rc = KSORT_OK;
  for (int r = 0; r < reps + 1 && rc == KSORT_OK; ++r) {
    KSORT_HIP(hipMemcpyAsync(work, src, (size_t)n * kb, hipMemcpyDeviceToDevice, st));
    KSORT_HIP(hipEventRecord(e0, st));
    rc = run_sort(dtype, work, n, nullptr, 1, nullptr, &tn, st, false);
    if (rc) break;
    KSORT_HIP(hipEventRecord(e1, st));
    KSORT_HIP(hipEventSynchronize(e1));
    float ms = 0.f;
    KSORT_HIP(hipEventElapsedTime(&ms, e0, e1));
    if (r > 0) best = std::min(best, (double)ms);  // first run warms up
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *best_ms = best;
  return rc;
}

}  // namespace ksort

using namespace ksort;

extern "C" {

int ksort_autotune(int dtype, int64_t n, ksort_tuning* out, void* stream) {
  if (dtype != KSORT_F64 && dtype != KSORT_F32) return fail(KSORT_EINVAL, "bad dtype");
  if (n < 2) return fail(KSORT_EINVAL, "autotune needs n >= 2");
  const size_t kb = dtype == KSORT_F64 ? 8 : 4;
  hipStream_t st = (hipStream_t)stream;
  void* src = nullptr;
  void* work = nullptr;
  KSORT_HIP(hipMalloc(&src, (size_t)n * kb));
  hipError_t e = hipMalloc(&work, (size_t)n * kb);
  if (e != hipSuccess) {
    (void)hipFree(src);
    return hip_fail(e, "hipMalloc(autotune)");
  }
  if (dtype == KSORT_F64)
    hipLaunchKernelGGL(fill_uniform<double>, dim3(1024), dim3(256), 0, st, (double*)src, n, 0x5EEDull);
  else
    hipLaunchKernelGGL(fill_uniform<float>, dim3(1024), dim3(256), 0, st, (float*)src, n, 0x5EEDull);
  int rc = KSORT_OK;
  ksort_tuning best{};
  double best_ms = 1e30;
  for (const auto& v : variants()) {
    if (v.dtype != dtype) continue;
    ksort_tuning tn{v.block, v.items, v.cutoff, 0};
    double ms = 0;
    rc = time_variant(dtype, tn, src, work, n, kb, st, 3, &ms);
    if (rc) break;
    if (ms < best_ms) {
      best_ms = ms;
      best = tn;
    }
  }
  (void)hipStreamSynchronize(st);
  (void)hipFree(src);
  (void)hipFree(work);
  if (rc) return rc;
  {
    std::lock_guard<std::mutex> lk(g_tuned_mu);
    g_tuned[{dtype, bucket_of(n)}] = best;
  }
  if (out) *out = best;
  return KSORT_OK;
}

}  // extern "C"
