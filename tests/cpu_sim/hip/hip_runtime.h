// Host build of the library for tests: a small HIP runtime on the CPU.
//
// The library's sources (host driver, server and kernels) compile unchanged
// against this header with g++.  Device memory is host memory with guard
// pages around every allocation, so an access out of bounds stops the test
// at once.  A kernel launch runs the grid on CPU threads, one per resident
// workgroup, in block order, each workgroup's threads as fibers that switch
// at barriers, cross-lane operations and s_sleep; cross-lane operations of a
// wave (ballot, readlane, readfirstlane, DPP row shifts and broadcasts) wait
// for all 64 lanes.  Every stream operation runs when it is enqueued (or is
// recorded while a stream captures a graph), so streams and events only keep
// their order.  Test use only; the product is built with hipcc for gfx950.
#pragma once

#include <stddef.h>
#include <stdint.h>
#include <string.h>

#include <functional>
#include <utility>

// ------------------------------------------------------------------ types
typedef int hipError_t;
enum : int {
  hipSuccess = 0,
  hipErrorInvalidValue = 1,
  hipErrorOutOfMemory = 2,
  hipErrorNotReady = 600,
  hipErrorUnknown = 999,
};
struct dim3 {
  unsigned x, y, z;
  dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {}
};
typedef struct ksim_stream* hipStream_t;
typedef struct ksim_event* hipEvent_t;
typedef struct ksim_graph* hipGraph_t;
typedef struct ksim_graph* hipGraphExec_t;
typedef struct ksim_graph_node* hipGraphNode_t;
struct hipDeviceProp_t {
  char name[256];
  char gcnArchName[256];
  int multiProcessorCount;
  size_t totalGlobalMem;
};
enum hipMemcpyKind { hipMemcpyHostToHost, hipMemcpyHostToDevice, hipMemcpyDeviceToHost, hipMemcpyDeviceToDevice, hipMemcpyDefault };
enum hipStreamCaptureMode { hipStreamCaptureModeGlobal, hipStreamCaptureModeThreadLocal, hipStreamCaptureModeRelaxed };
#define hipStreamDefault 0
#define hipStreamNonBlocking 1
#define hipEventDefault 0
#define hipEventDisableTiming 2
#define hipHostMallocDefault 0

// ------------------------------------------------------------------ host API
hipError_t hipMalloc(void** p, size_t bytes);
hipError_t hipFree(void* p);
hipError_t hipHostMalloc(void** p, size_t bytes, unsigned flags);
hipError_t hipHostFree(void* p);
hipError_t hipMemcpy(void* dst, const void* src, size_t bytes, hipMemcpyKind kind);
hipError_t hipMemcpyAsync(void* dst, const void* src, size_t bytes, hipMemcpyKind kind, hipStream_t s);
hipError_t hipMemsetAsync(void* dst, int value, size_t bytes, hipStream_t s);
hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned flags);
hipError_t hipStreamDestroy(hipStream_t s);
hipError_t hipStreamSynchronize(hipStream_t s);
hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned flags);
hipError_t hipEventCreate(hipEvent_t* e);
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned flags);
hipError_t hipEventDestroy(hipEvent_t e);
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s);
hipError_t hipEventSynchronize(hipEvent_t e);
hipError_t hipEventElapsedTime(float* ms, hipEvent_t a, hipEvent_t b);
hipError_t hipGetDevice(int* d);
hipError_t hipSetDevice(int d);
hipError_t hipGetDeviceCount(int* n);
hipError_t hipGetDeviceProperties(hipDeviceProp_t* p, int d);
hipError_t hipOccupancyMaxActiveBlocksPerMultiprocessor(int* n, const void* f, int block, size_t shmem);
hipError_t hipGetLastError();
const char* hipGetErrorString(hipError_t e);
hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode m);
hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t* g);
hipError_t hipGraphInstantiate(hipGraphExec_t* e, hipGraph_t g, hipGraphNode_t* err, char* log, size_t n);
hipError_t hipGraphDestroy(hipGraph_t g);
hipError_t hipGraphExecDestroy(hipGraphExec_t e);
hipError_t hipGraphLaunch(hipGraphExec_t e, hipStream_t s);

// Runs `body` for every thread of the grid (or records it in a capture).
void ksim_launch(hipStream_t s, dim3 grid, dim3 block, std::function<void()> body);

template <typename F, typename... A>
void ksim_launch_args(hipStream_t s, dim3 grid, dim3 block, F f, A... a) {
  ksim_launch(s, grid, block, [f, a...]() { f(a...); });
}
#define hipLaunchKernelGGL(kernel, grid, block, shmem, stream, ...) \
  ksim_launch_args((stream), dim3(grid), dim3(block), (kernel), __VA_ARGS__)

// ------------------------------------------------------------------ device side
#define __global__
#define __device__
#define __host__
#define __forceinline__ inline
#define __launch_bounds__(...)
#define __shared__ static thread_local  // one CPU thread runs one workgroup at a time
#define __align__(n) __attribute__((aligned(n)))
#define HIP_SYMBOL(x) (&(x))
hipError_t hipGetSymbolAddress(void** p, const void* symbol);

struct ksim_dims {
  dim3 tid, bid, bdim, gdim;
};
ksim_dims* ksim_cur();
#define threadIdx (ksim_cur()->tid)
#define blockIdx (ksim_cur()->bid)
#define blockDim (ksim_cur()->bdim)
#define gridDim (ksim_cur()->gdim)

void __syncthreads();
// 1 if any thread of the workgroup passes a nonzero value (a barrier)
inline int __syncthreads_or(int p) {
  static thread_local int acc;
  __syncthreads();  // every thread has read the previous result
  if (ksim_cur()->tid.x == 0) acc = 0;
  __syncthreads();
  if (p) acc = 1;
  __syncthreads();
  return acc;
}
void ksim_yield();
uint64_t ksim_ballot(bool pred);
uint32_t ksim_lane();
// value of lane `src` of the wave, for every lane (a collective)
uint64_t ksim_readlane(uint64_t v, int src);
uint64_t ksim_readfirstlane(uint64_t v);
int ksim_dpp(int old, int v, int ctrl, int row_mask, int bank_mask, bool bound_ctrl);

// value of lane `src` (its own choice per lane) of the wave (a collective)
uint64_t ksim_shfl(uint64_t v, int src);

inline uint64_t __ballot(int pred) { return ksim_ballot(pred != 0); }
template <typename T>
inline T __shfl(T v, int src, int width = 64) {
  static_assert(sizeof(T) <= 8, "__shfl of a value wider than 8 bytes");
  uint64_t b = 0;
  memcpy(&b, &v, sizeof(T));
  const int base = (int)ksim_lane() / width * width;
  b = ksim_shfl(b, base + ((src % width) + width) % width);
  T r;
  memcpy(&r, &b, sizeof(T));
  return r;
}
template <typename T>
inline T __shfl_xor(T v, int mask, int width = 64) {
  return __shfl(v, (int)ksim_lane() ^ mask, width);
}
template <typename T>
inline T __shfl_up(T v, unsigned d, int width = 64) {
  const int l = (int)ksim_lane(), src = l - (int)d;
  return __shfl(v, src >= l / width * width ? src : l, width);
}
inline int __popcll(unsigned long long x) { return __builtin_popcountll(x); }
#define __builtin_amdgcn_readfirstlane(v) ((int)ksim_readfirstlane((uint64_t)(uint32_t)(v)))
#define __builtin_amdgcn_readlane(v, j) ((int)ksim_readlane((uint64_t)(uint32_t)(v), (j)))
#define __builtin_amdgcn_update_dpp(old, v, ctrl, rm, bm, bc) ksim_dpp((old), (v), (ctrl), (rm), (bm), (bc))
#define __builtin_amdgcn_s_sleep(n) ksim_yield()
inline uint32_t ksim_mbcnt_lo(uint32_t m, uint32_t acc) {
  const uint32_t l = ksim_lane();
  return acc + (uint32_t)__builtin_popcount(l >= 32 ? m : (m & ((1u << l) - 1)));
}
inline uint32_t ksim_mbcnt_hi(uint32_t m, uint32_t acc) {
  const uint32_t l = ksim_lane();
  return acc + (uint32_t)__builtin_popcount(l < 32 ? 0u : (m & ((1u << (l - 32)) - 1)));
}
#define __builtin_amdgcn_mbcnt_lo(m, acc) ksim_mbcnt_lo((m), (acc))
#define __builtin_amdgcn_mbcnt_hi(m, acc) ksim_mbcnt_hi((m), (acc))

#define __HIP_MEMORY_SCOPE_WORKGROUP 1
#define __HIP_MEMORY_SCOPE_AGENT 2
#define __HIP_MEMORY_SCOPE_SYSTEM 3
#define __hip_atomic_load(p, order, scope) __atomic_load_n((p), __ATOMIC_SEQ_CST)
#define __hip_atomic_store(p, v, order, scope) __atomic_store_n((p), (v), __ATOMIC_SEQ_CST)
#define __hip_atomic_fetch_add(p, v, order, scope) __atomic_fetch_add((p), (v), __ATOMIC_SEQ_CST)

inline int atomicAdd(int* p, int v) { return __atomic_fetch_add(p, v, __ATOMIC_SEQ_CST); }
inline unsigned atomicAdd(unsigned* p, unsigned v) { return __atomic_fetch_add(p, v, __ATOMIC_SEQ_CST); }
inline unsigned long long atomicAdd(unsigned long long* p, unsigned long long v) {
  return __atomic_fetch_add(p, v, __ATOMIC_SEQ_CST);
}

// the device-side min and max of HIP
inline int min(int a, int b) { return a < b ? a : b; }
inline int max(int a, int b) { return a > b ? a : b; }
inline long long min(long long a, long long b) { return a < b ? a : b; }
inline long long max(long long a, long long b) { return a > b ? a : b; }
inline long min(long a, long b) { return a < b ? a : b; }
inline long max(long a, long b) { return a > b ? a : b; }
inline int atomicExch(int* p, int v) { return __atomic_exchange_n(p, v, __ATOMIC_SEQ_CST); }
inline int atomicOr(int* p, int v) { return __atomic_fetch_or(p, v, __ATOMIC_SEQ_CST); }
inline int atomicCAS(int* p, int cmp, int v) {
  __atomic_compare_exchange_n(p, &cmp, v, false, __ATOMIC_SEQ_CST, __ATOMIC_SEQ_CST);
  return cmp;
}
inline int atomicMax(int* p, int v) {
  int old = __atomic_load_n(p, __ATOMIC_SEQ_CST);
  while (old < v && !__atomic_compare_exchange_n(p, &old, v, false, __ATOMIC_SEQ_CST, __ATOMIC_SEQ_CST)) {
  }
  return old;
}

struct int2 {
  int x, y;
};
struct alignas(16) int4 {
  int x, y, z, w;
};
inline int2 make_int2(int x, int y) { return int2{x, y}; }
inline int4 make_int4(int x, int y, int z, int w) { return int4{x, y, z, w}; }

inline float __int_as_float(int x) {
  float f;
  memcpy(&f, &x, 4);
  return f;
}
inline int __float_as_int(float f) {
  int x;
  memcpy(&x, &f, 4);
  return x;
}
inline double __longlong_as_double(long long x) {
  double d;
  memcpy(&d, &x, 8);
  return d;
}
inline long long __double_as_longlong(double d) {
  long long x;
  memcpy(&x, &d, 8);
  return x;
}

// The kernels' inline-assembly helpers, as host code.
// Lanes of a wave run one after another here, so the points where the
// kernels rely on a wave executing in step (an LDS wait, a marked step)
// wait for every lane of the wave.
void ksim_wave_sync();
#define KS_OPAQUE(x) asm volatile("" : "+m"(x))
#define KS_LDS_WAIT() ksim_wave_sync()
#define KS_MEM_FENCE() asm volatile("" ::: "memory")
#define KS_WAVE_STEP() ksim_wave_sync()
// 16-byte vectors of keys (the kernels' KeyVec), as plain structs
#define KS_KEY_VEC_DEFINED
namespace ksort {
template <typename T>
struct KeyVec {
  struct type {
    T e[16 / sizeof(T)];
    T operator[](int i) const { return e[i]; }
  };
};
}  // namespace ksort
