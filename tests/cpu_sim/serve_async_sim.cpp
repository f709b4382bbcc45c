// The serving workload's host-side pattern on the host build with
// asynchronous in-order queues (run with KSIM_HWQ=Q): plain sorts on the null
// stream first; then a producer stream that draws each request's keys with a
// kernel and synchronizes before submitting it; a checker thread that waits
// for the requests in order, runs a check kernel on a stream of its own,
// copies its verdict back and returns the buffer to a pool that later
// requests reuse (as a caching allocator does).  Every request's keys are
// compared with std::sort and its first pivot with the count of smaller keys.
//
//   serve_async_sim COUNT LO HI INFLIGHT BUDGET_MIB PACE_US
#include <unistd.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "hip/hip_runtime.h"
#include "ksort.h"

static __host__ __device__ uint64_t mix(uint64_t seed, uint64_t t) {
  uint64_t z = seed + (t + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
static double u01(uint64_t seed, uint64_t t) { return (double)(mix(seed, t) >> 11) * 0x1p-53; }

template <typename T>
__global__ void fill_kernel(T* out, int64_t n, uint64_t seed) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t z = mix(seed, (uint64_t)t);
    out[t] = sizeof(T) == 8 ? (T)((double)(z >> 11) * 0x1p-53) : (T)((double)(z >> 40) * 0x1p-24);
  }
}

template <typename T>
__global__ void check_kernel(const T* a, int64_t n, int* bad) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t + 1 < n; t += (int64_t)gridDim.x * blockDim.x)
    if (a[t + 1] < a[t]) atomicAdd(bad, 1);
}

template <typename T>
static void host_keys(int64_t n, uint64_t seed, std::vector<T>& a) {
  a.resize(n);
  for (int64_t t = 0; t < n; ++t) {
    const uint64_t z = mix(seed, (uint64_t)t);
    a[t] = sizeof(T) == 8 ? (T)((double)(z >> 11) * 0x1p-53) : (T)((double)(z >> 40) * 0x1p-24);
  }
}

struct Req {
  int64_t n = 0;
  bool f64 = true;
  void* d = nullptr;
  size_t cap = 0;
  uint64_t ticket = 0;
  std::atomic<bool> submitted{false};
};

static std::mutex pool_mu;
static std::multimap<size_t, void*> pool;  // freed buffers by capacity

static void* take(size_t bytes, size_t* cap) {
  const size_t c = (bytes + (2u << 20) - 1) / (2u << 20) * (2u << 20);
  {
    std::lock_guard<std::mutex> lk(pool_mu);
    auto it = pool.lower_bound(c);
    if (it != pool.end() && it->first < 2 * c) {
      void* p = it->second;
      *cap = it->first;
      pool.erase(it);
      return p;
    }
  }
  void* p = nullptr;
  hipMalloc(&p, c);
  *cap = c;
  return p;
}
static void give(void* p, size_t cap) {
  std::lock_guard<std::mutex> lk(pool_mu);
  pool.emplace(cap, p);
}

template <typename T>
static bool verify(const Req& q, uint64_t seed, int64_t pivot, hipStream_t st, const char** why) {
  int* d_bad = nullptr;
  hipMalloc((void**)&d_bad, sizeof(int));
  int h_bad = 0;
  hipMemcpyAsync(d_bad, &h_bad, sizeof(int), hipMemcpyHostToDevice, st);
  hipLaunchKernelGGL(check_kernel<T>, dim3((unsigned)std::min<int64_t>(64, (q.n + 255) / 256)), dim3(256), 0, st,
                     (const T*)q.d, q.n, d_bad);
  hipMemcpyAsync(&h_bad, d_bad, sizeof(int), hipMemcpyDeviceToHost, st);
  hipStreamSynchronize(st);
  std::vector<T> a, got(q.n);
  host_keys<T>(q.n, seed, a);
  hipMemcpyAsync(got.data(), q.d, q.n * sizeof(T), hipMemcpyDeviceToHost, st);
  hipStreamSynchronize(st);
  int64_t fp = 0;
  for (int64_t t = 1; t < q.n; ++t) fp += !(a[0] <= a[t]);
  std::sort(a.begin(), a.end());
  if (h_bad != 0) *why = "check kernel found descents";
  else if (memcmp(got.data(), a.data(), q.n * sizeof(T)) != 0) *why = "keys differ from std::sort";
  else if (pivot != fp) *why = "first pivot differs from the count of smaller keys";
  else return true;
  return false;
}

int main(int argc, char** argv) {
  setvbuf(stdout, nullptr, _IONBF, 0);
  const int count = argc > 1 ? atoi(argv[1]) : 300;
  const double lo = argc > 2 ? atof(argv[2]) : 1e3, hi = argc > 3 ? atof(argv[3]) : 3e4;
  const int inflight = argc > 4 ? atoi(argv[4]) : 256;
  const size_t budget = (size_t)(argc > 5 ? atol(argv[5]) : 1024) << 20;
  const int pace_us = argc > 6 ? atoi(argv[6]) : 200;
  // plain sorts on the null stream first
  for (int k = 0; k < 20; ++k) {
    const int64_t n = 1000 + 7919 * k;
    double* d = nullptr;
    hipMalloc((void**)&d, n * 8);
    hipLaunchKernelGGL(fill_kernel<double>, dim3(16), dim3(256), 0, nullptr, d, n, (uint64_t)(77 + k));
    if (ksort_f64(d, n, nullptr) != KSORT_OK) {
      printf("plain sort failed: %s\n", ksort_last_error());
      return 1;
    }
    give(d, n * 8);
  }
  hipStream_t prod, chk;
  hipStreamCreateWithFlags(&prod, hipStreamNonBlocking);
  hipStreamCreateWithFlags(&chk, hipStreamNonBlocking);
  ksort_server* srv = ksort_server_create(budget, inflight, 0);
  if (!srv) {
    printf("server_create failed: %s\n", ksort_last_error());
    return 1;
  }
  std::vector<Req> reqs(count);
  for (int r = 0; r < count; ++r) {
    const double u = u01(12, r);
    reqs[r].n = std::min<int64_t>((int64_t)hi, std::max<int64_t>((int64_t)lo, (int64_t)std::floor(std::exp(std::log(lo) + u * (std::log(hi) - std::log(lo))))));
    reqs[r].f64 = u01(13, r) < 0.7;
  }
  printf("serve async sim: %d requests, sizes [%g, %g], %d in flight\n", count, lo, hi, inflight);
  std::atomic<int> wrong{0};
  std::thread checker([&]() {
    for (int r = 0; r < count; ++r) {
      while (!reqs[r].submitted.load()) std::this_thread::yield();
      const int rc = ksort_server_wait(srv, reqs[r].ticket, 60.0);
      if (rc != KSORT_OK) {
        ksort_server_stats_t st;
        ksort_server_stats(srv, &st);
        printf("request %d (n=%lld): wait returned %d (%s); completed %lld, in flight %lld, queued %lld, ticks %lld\n",
               r, (long long)reqs[r].n, rc, ksort_last_error(), (long long)st.completed, (long long)st.inflight_now,
               (long long)st.queued_now, (long long)st.ticks);
        _exit(3);
      }
      ksort_request_info info;
      ksort_server_result(srv, reqs[r].ticket, &info);
      const char* why = "";
      const uint64_t seed = 1000000 + r;
      const bool ok = reqs[r].f64 ? verify<double>(reqs[r], seed, info.first_pivot, chk, &why)
                                  : verify<float>(reqs[r], seed, info.first_pivot, chk, &why);
      if (!ok) {
        printf("request %d (n=%lld %s): %s\n", r, (long long)reqs[r].n, reqs[r].f64 ? "f64" : "f32", why);
        ++wrong;
      }
      give(reqs[r].d, reqs[r].cap);
      if (r % 100 == 99) printf("  %d checked\n", r + 1);
    }
  });
  for (int r = 0; r < count; ++r) {
    Req& q = reqs[r];
    q.d = take(q.n * (q.f64 ? 8 : 4), &q.cap);
    const unsigned g = (unsigned)std::min<int64_t>(64, (q.n + 255) / 256);
    if (q.f64)
      hipLaunchKernelGGL(fill_kernel<double>, dim3(g), dim3(256), 0, prod, (double*)q.d, q.n, (uint64_t)(1000000 + r));
    else
      hipLaunchKernelGGL(fill_kernel<float>, dim3(g), dim3(256), 0, prod, (float*)q.d, q.n, (uint64_t)(1000000 + r));
    hipStreamSynchronize(prod);
    if (ksort_server_submit(srv, q.f64 ? KSORT_F64 : KSORT_F32, q.d, q.n, &q.ticket) != KSORT_OK) {
      printf("submit %d failed: %s\n", r, ksort_last_error());
      _exit(2);
    }
    q.submitted.store(true);
    if (pace_us > 0) std::this_thread::sleep_for(std::chrono::microseconds(pace_us));
  }
  checker.join();
  ksort_server_stats_t st;
  ksort_server_stats(srv, &st);
  printf("serve async sim: %lld completed, %lld failed, %lld ticks, %d wrong\n", (long long)st.completed,
         (long long)st.failed, (long long)st.ticks, wrong.load());
  ksort_server_destroy(srv);
  return wrong.load() == 0 && st.completed == count ? 0 : 1;
}
