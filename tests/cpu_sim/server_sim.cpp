// The sort server on the host build: a stream of requests of mixed sizes
// and key types, submitted at a steady pace while a second thread waits for
// them in order, checks each result (sorted like std::sort, first pivot
// equal to the count of keys smaller than the first) and frees it, so that
// request slots, scratch ranges and buffers are reused many times over.
// A request that does not complete within the wait limit ends the run with
// the server's counters printed.
//
//   server_sim COUNT LO HI INFLIGHT BUDGET_MIB PACE_US
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <thread>
#include <vector>

#include <unistd.h>

#include "hip/hip_runtime.h"
#include "ksort.h"

static uint64_t mix(uint64_t seed, uint64_t t) {
  uint64_t z = seed + (t + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
static double u01(uint64_t seed, uint64_t t) { return (double)(mix(seed, t) >> 11) * 0x1p-53; }

struct Req {
  int64_t n = 0;
  bool f64 = true;
  void* d = nullptr;
  uint64_t ticket = 0;
  std::atomic<bool> submitted{false};
};

template <typename T>
static bool check(const Req& q, int64_t seed, int64_t pivot, const char** why) {
  std::vector<T> a(q.n), got(q.n);
  for (int64_t t = 0; t < q.n; ++t)
    a[t] = sizeof(T) == 8 ? (T)u01(seed, t) : (T)((double)(mix(seed, t) >> 40) * 0x1p-24);
  hipMemcpy(got.data(), q.d, q.n * sizeof(T), hipMemcpyDeviceToHost);
  int64_t fp = 0;
  for (int64_t t = 1; t < q.n; ++t) fp += !(a[0] <= a[t]);
  std::vector<T> want = a;
  std::sort(want.begin(), want.end());
  if (memcmp(got.data(), want.data(), q.n * sizeof(T)) != 0) {
    *why = "keys differ from std::sort";
    return false;
  }
  if (pivot != fp) {
    *why = "first pivot differs from the count of smaller keys";
    return false;
  }
  return true;
}

template <typename T>
static void fill(const Req& q, int64_t seed) {
  std::vector<T> a(q.n);
  for (int64_t t = 0; t < q.n; ++t)
    a[t] = sizeof(T) == 8 ? (T)u01(seed, t) : (T)((double)(mix(seed, t) >> 40) * 0x1p-24);
  hipMemcpy(q.d, a.data(), q.n * sizeof(T), hipMemcpyHostToDevice);
}

int main(int argc, char** argv) {
  setvbuf(stdout, nullptr, _IONBF, 0);
  const int count = argc > 1 ? atoi(argv[1]) : 300;
  const double lo = argc > 2 ? atof(argv[2]) : 1e3, hi = argc > 3 ? atof(argv[3]) : 3e4;
  const int inflight = argc > 4 ? atoi(argv[4]) : 256;
  const size_t budget = (size_t)(argc > 5 ? atol(argv[5]) : 1024) << 20;
  const int pace_us = argc > 6 ? atoi(argv[6]) : 200;
  ksort_server* srv = ksort_server_create(budget, inflight, 0);
  if (!srv) {
    printf("server_create failed: %s\n", ksort_last_error());
    return 1;
  }
  std::vector<Req> reqs(count);
  int64_t keys = 0;
  for (int r = 0; r < count; ++r) {
    const double u = u01(12, r);
    reqs[r].n = std::min<int64_t>((int64_t)hi, std::max<int64_t>((int64_t)lo, (int64_t)std::floor(std::exp(std::log(lo) + u * (std::log(hi) - std::log(lo))))));
    reqs[r].f64 = u01(13, r) < 0.7;
    keys += reqs[r].n;
  }
  printf("server sim: %d requests, %lld keys, sizes [%g, %g], %d in flight, %zu MiB\n", count, (long long)keys, lo, hi,
         inflight, budget >> 20);
  std::atomic<int> failures{0};
  std::thread checker([&]() {
    for (int r = 0; r < count; ++r) {
      while (!reqs[r].submitted.load()) std::this_thread::yield();
      const int rc = ksort_server_wait(srv, reqs[r].ticket, 120.0);
      if (rc != KSORT_OK) {
        ksort_server_stats_t st;
        ksort_server_stats(srv, &st);
        printf("request %d (n=%lld %s): wait returned %d (%s); completed %lld, failed %lld, in flight %lld, "
               "queued %lld, ticks %lld\n",
               r, (long long)reqs[r].n, reqs[r].f64 ? "f64" : "f32", rc, ksort_last_error(), (long long)st.completed,
               (long long)st.failed, (long long)st.inflight_now, (long long)st.queued_now, (long long)st.ticks);
        fflush(stdout);
        _exit(3);
      }
      ksort_request_info info;
      ksort_server_result(srv, reqs[r].ticket, &info);
      const char* why = "";
      const int64_t seed = 1000000 + r;
      const bool ok = reqs[r].f64 ? check<double>(reqs[r], seed, info.first_pivot, &why)
                                  : check<float>(reqs[r], seed, info.first_pivot, &why);
      if (!ok) {
        printf("request %d (n=%lld %s): %s\n", r, (long long)reqs[r].n, reqs[r].f64 ? "f64" : "f32", why);
        ++failures;
      }
      hipFree(reqs[r].d);
      reqs[r].d = nullptr;
      if (r % 100 == 99) printf("  %d checked\n", r + 1);
    }
  });
  for (int r = 0; r < count; ++r) {
    Req& q = reqs[r];
    hipMalloc(&q.d, q.n * (q.f64 ? 8 : 4));
    if (q.f64)
      fill<double>(q, 1000000 + r);
    else
      fill<float>(q, 1000000 + r);
    const int rc = ksort_server_submit(srv, q.f64 ? KSORT_F64 : KSORT_F32, q.d, q.n, &q.ticket);
    if (rc != KSORT_OK) {
      printf("submit %d failed %d: %s\n", r, rc, ksort_last_error());
      _exit(2);
    }
    q.submitted.store(true);
    if (pace_us > 0) std::this_thread::sleep_for(std::chrono::microseconds(pace_us));
  }
  checker.join();
  ksort_server_stats_t st;
  ksort_server_stats(srv, &st);
  printf("server sim: %lld completed, %lld failed, %lld ticks, %d wrong\n", (long long)st.completed,
         (long long)st.failed, (long long)st.ticks, failures.load());
  ksort_server_destroy(srv);
  return failures.load() == 0 && st.completed == count ? 0 : 1;
}
