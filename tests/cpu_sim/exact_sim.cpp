// Host build run of the literal arrangement (Steps 1-4 as the sequential
// steps leave the array) against the C oracle, which this test program links:
//  * one level on many disjoint segments (with gaps): every pivot index and
//    every position inside the segments equal the oracle's, positions
//    outside keep the sentinel the output buffer started with;
//  * the whole sort: the final array, the first pivot and the set of calls
//    (left, right, i) equal the oracle's.
// Key kinds: uniform, eight distinct values, ascending, all equal, organ
// pipe; both key widths.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "hip/hip_runtime.h"
#include "ksort.h"
#include "ksort_oracle.h"

static uint64_t mix(uint64_t seed, uint64_t t) {
  uint64_t z = seed + (t + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

static std::vector<double> make_keys(int kind, uint64_t seed, long n) {
  std::vector<double> a(n);
  for (long t = 0; t < n; ++t) a[t] = (double)(mix(seed, t) >> 11) * 0x1p-53;
  if (kind == 1)
    for (auto& x : a) x = std::floor(x * 8);
  if (kind == 2) std::sort(a.begin(), a.end());
  if (kind == 3)
    for (auto& x : a) x = 0.25;
  if (kind == 4)
    for (long t = 0; t < n; ++t) a[t] = (double)(t < n / 2 ? t : n - 1 - t);
  return a;
}

template <typename T>
struct Oracle;
template <>
struct Oracle<double> {
  static int sort(double* a, int64_t n, int64_t* fp, ksort_oracle_call* tr, int64_t cap, int64_t* nc) {
    return ksort_oracle_sort_f64(a, n, fp, tr, cap, nc, nullptr);
  }
  static int level(double* a, const int64_t* l, const int64_t* len, int64_t ns, int64_t* p) {
    return ksort_oracle_partition_level_f64(a, l, len, ns, p);
  }
  static constexpr int dtype = KSORT_F64;
};
template <>
struct Oracle<float> {
  static int sort(float* a, int64_t n, int64_t* fp, ksort_oracle_call* tr, int64_t cap, int64_t* nc) {
    return ksort_oracle_sort_f32(a, n, fp, tr, cap, nc, nullptr);
  }
  static int level(float* a, const int64_t* l, const int64_t* len, int64_t ns, int64_t* p) {
    return ksort_oracle_partition_level_f32(a, l, len, ns, p);
  }
  static constexpr int dtype = KSORT_F32;
};

template <typename T>
static bool bit_equal(const std::vector<T>& x, const std::vector<T>& y) {
  return x.size() == y.size() && std::memcmp(x.data(), y.data(), x.size() * sizeof(T)) == 0;
}

template <typename T, typename P>
static P* to_dev(const std::vector<T>& h) {
  void* d = nullptr;
  hipMalloc(&d, std::max<size_t>(1, h.size()) * sizeof(T));
  if (!h.empty()) hipMemcpy(d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice);
  return (P*)d;
}

template <typename T>
static std::vector<T> to_host(const void* d, size_t n) {
  std::vector<T> h(n);
  if (n) hipMemcpy(h.data(), d, n * sizeof(T), hipMemcpyDeviceToHost);
  return h;
}

template <typename T>
static int check_sort(int kind, long n) {
  const std::vector<double> k64 = make_keys(kind, 11 + n, n);
  std::vector<T> a(k64.begin(), k64.end());
  std::vector<T> want = a;
  int64_t ncalls = 0, wfp = 0;
  Oracle<T>::sort(want.data(), n, &wfp, nullptr, 0, &ncalls);
  std::vector<ksort_oracle_call> tr((size_t)std::max<int64_t>(ncalls, 1));
  std::vector<T> again = a;
  Oracle<T>::sort(again.data(), n, nullptr, tr.data(), ncalls, nullptr);
  std::vector<std::array<int64_t, 3>> wc;
  for (int64_t j = 0; j < ncalls; ++j) wc.push_back({tr[j].left, tr[j].right, tr[j].i});
  std::sort(wc.begin(), wc.end());

  T* d = to_dev<T, T>(a);
  int64_t *dfp = nullptr, *dcalls = nullptr, *dn = nullptr;
  hipMalloc((void**)&dfp, 8);
  hipMalloc((void**)&dcalls, (size_t)std::max<int64_t>(ncalls, 1) * 3 * 8);
  hipMalloc((void**)&dn, 8);
  const int rc = ksort_sort_exact(Oracle<T>::dtype, d, n, dfp, dcalls, std::max<int64_t>(ncalls, 1), dn, nullptr);
  if (rc) {
    printf("sort_exact failed %d: %s\n", rc, ksort_last_error());
    return 1;
  }
  const std::vector<T> got = to_host<T>(d, n);
  const int64_t gfp = to_host<int64_t>(dfp, 1)[0], gn = to_host<int64_t>(dn, 1)[0];
  const std::vector<int64_t> gcf = to_host<int64_t>(dcalls, (size_t)std::max<int64_t>(gn, 0) * 3);
  std::vector<std::array<int64_t, 3>> gc;
  for (int64_t j = 0; j < gn && j < ncalls; ++j) gc.push_back({gcf[3 * j], gcf[3 * j + 1], gcf[3 * j + 2]});
  std::sort(gc.begin(), gc.end());
  const bool ok = bit_equal(got, want) && gfp == wfp && gn == ncalls && gc == wc;
  printf("sort_exact %s n=%ld kind=%d: %s (calls %lld / %lld, first pivot %lld / %lld)\n",
         sizeof(T) == 8 ? "f64" : "f32", n, kind, ok ? "ok" : "MISMATCH", (long long)gn, (long long)ncalls,
         (long long)gfp, (long long)wfp);
  hipFree(d);
  hipFree(dfp);
  hipFree(dcalls);
  hipFree(dn);
  return ok ? 0 : 1;
}

template <typename T>
static int check_level(int kind, long n, long maxlen, uint64_t seed) {
  const std::vector<double> k64 = make_keys(kind, seed, n);
  std::vector<T> a(k64.begin(), k64.end());
  std::vector<int64_t> left, len;
  long pos = 0;
  for (uint64_t t = 0;; ++t) {
    pos += (long)(mix(seed + 1, t) % 64);
    // log-uniform length in [1, maxlen]
    const double u = (double)(mix(seed + 2, t) >> 11) * 0x1p-53;
    const long L = std::max(1L, std::min(maxlen, (long)std::exp(u * std::log((double)maxlen + 1))));
    if (pos + L > n) break;
    left.push_back(pos);
    len.push_back(L);
    pos += L;
  }
  std::vector<T> want = a;
  std::vector<int64_t> wp(left.size());
  Oracle<T>::level(want.data(), left.data(), len.data(), (int64_t)left.size(), wp.data());

  const T sentinel = (T)-7;
  T* din = to_dev<T, T>(a);
  T* dout = to_dev<T, T>(std::vector<T>(n, sentinel));
  int64_t* dl = to_dev<int64_t, int64_t>(left);
  int64_t* dlen = to_dev<int64_t, int64_t>(len);
  int64_t* dp = to_dev<int64_t, int64_t>(std::vector<int64_t>(left.size(), -1));
  const int rc = ksort_partition_level_exact(Oracle<T>::dtype, din, dout, n, dl, dlen, (int64_t)left.size(), dp, nullptr);
  if (rc) {
    printf("level_exact failed %d: %s\n", rc, ksort_last_error());
    return 1;
  }
  const std::vector<T> got = to_host<T>(dout, n);
  const std::vector<int64_t> gp = to_host<int64_t>(dp, left.size());
  std::vector<char> covered(n, 0);
  for (size_t s = 0; s < left.size(); ++s)
    for (long x = left[s]; x < left[s] + len[s]; ++x) covered[x] = 1;
  long bad = 0;
  for (long x = 0; x < n; ++x) {
    const T w = covered[x] ? want[x] : sentinel;
    if (std::memcmp(&got[x], &w, sizeof(T)) != 0) ++bad;
  }
  const bool ok = bad == 0 && gp == wp;
  printf("level_exact %s n=%ld nseg=%zu kind=%d: %s (%ld positions differ)\n", sizeof(T) == 8 ? "f64" : "f32", n,
         left.size(), kind, ok ? "ok" : "MISMATCH", bad);
  hipFree(din);
  hipFree(dout);
  hipFree(dl);
  hipFree(dlen);
  hipFree(dp);
  return ok ? 0 : 1;
}

int main(int argc, char** argv) {
  setvbuf(stdout, nullptr, _IONBF, 0);
  int fails = 0;
  // arguments: pairs of n and the key kinds to sort at that n (digits 0-4)
  for (int j = 1; j + 1 < argc; j += 2) {
    const long n = atol(argv[j]);
    for (const char* k = argv[j + 1]; *k; ++k) {
      const int kind = *k - '0';
      fails += check_sort<double>(kind, n);
      if (kind < 2) fails += check_sort<float>(kind, n);
    }
    fails += check_level<double>(0, n, std::max(2L, n / 3), 5 + n);
    fails += check_level<double>(1, n, 40, 6 + n);
    fails += check_level<float>(0, n, std::max(2L, n / 7), 7 + n);
  }
  printf("%d failed\n", fails);
  return fails ? 1 : 0;
}
