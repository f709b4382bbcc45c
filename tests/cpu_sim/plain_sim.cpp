// Sanity run of the host build: plain sorts against std::sort (first pivot
// by its closed form), then exit.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "hip/hip_runtime.h"
#include "ksort.h"

static uint64_t mix(uint64_t seed, uint64_t t) {
  uint64_t z = seed + (t + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

int main(int argc, char** argv) {
  setvbuf(stdout, nullptr, _IONBF, 0);
  const long n = argc > 1 ? atol(argv[1]) : 100000;
  std::vector<double> a(n);
  for (long t = 0; t < n; ++t) a[t] = (double)(mix(5, t) >> 11) * 0x1p-53;
  double* d = nullptr;
  int64_t* fp = nullptr;
  hipMalloc((void**)&d, n * sizeof(double));
  hipMalloc((void**)&fp, sizeof(int64_t));
  hipMemcpy(d, a.data(), n * sizeof(double), hipMemcpyHostToDevice);
  int rc = ksort_sort_ex(KSORT_F64, d, n, fp, nullptr, nullptr);
  if (rc) {
    printf("sort failed %d: %s\n", rc, ksort_last_error());
    return 1;
  }
  std::vector<double> got(n);
  hipMemcpy(got.data(), d, n * sizeof(double), hipMemcpyDeviceToHost);
  int64_t gfp = 0;
  hipMemcpy(&gfp, fp, 8, hipMemcpyDeviceToHost);
  int64_t want_fp = 0;
  for (long t = 1; t < n; ++t) want_fp += !(a[0] <= a[t]);
  std::vector<double> want = a;
  std::sort(want.begin(), want.end());
  const bool ok = got == want && gfp == want_fp;
  if (!ok) {
    std::vector<double> g2 = got;
    std::sort(g2.begin(), g2.end());
    long bad = 0, first = -1;
    for (long t = 0; t < n; ++t)
      if (got[t] != want[t]) {
        if (first < 0) first = t;
        ++bad;
      }
    printf("  %ld positions differ, first %ld; output is %s permutation\n", bad, first, g2 == want ? "a" : "NOT a");
  }
  printf("plain n=%ld: %s (first pivot %lld, want %lld)\n", n, ok ? "ok" : "MISMATCH", (long long)gfp,
         (long long)want_fp);
  return ok ? 0 : 1;
}
