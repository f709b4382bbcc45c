// Autotuner: times every compiled kernel variant (threads per workgroup,
// keys per thread in a partition tile, LDS-finish cutoff) on an input of
// the requested shape and key type, and makes the fastest the variant used
// for inputs of about that size: single arrays (seeded U[0,1) keys of n) or
// packed batches (the caller's own batch).  A choice applies to its
// power-of-two size bucket, or the nearest tuned bucket at most two powers of
// two away.
//
// Choices persist in a JSON file keyed by (device architecture, kind, key
// type, size bucket), one entry per line:
//   {"version": 1, "entries": [
//   {"arch": "gfx950", "kind": "single", "dtype": 0, "bucket": 22, "block": 512, "items": 24, "cutoff": 2048,
//    "ms": 1.0125, "default_ms": 1.0200},
//   ...]}
// ksort_tune_file names the file (KSORT_TUNE_FILE does too, read at first
// use): its entries for the current device's architecture are applied, and
// every later tuning rewrites it.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
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

struct TuneEntry {
  std::string arch;
  int kind = kTuneSingle;
  int dtype = 0;
  int bucket = 0;
  ksort_tuning tn{};
  double ms = 0, default_ms = 0;
};

static std::mutex g_tuned_mu;
static std::vector<TuneEntry> g_entries;  // every entry known (all architectures)
static std::string g_tune_path;            // file the entries persist in ("" = none)
static bool g_env_checked = false;

static int bucket_of(int64_t n) { return n <= 1 ? 0 : (int)std::floor(std::log2((double)n)); }

static const char* kind_name(int kind) { return kind == kTuneBatch ? "batch" : "single"; }

static std::string device_arch() {
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return "";
  std::string a = prop.gcnArchName;
  const size_t c = a.find(':');
  return c == std::string::npos ? a : a.substr(0, c);
}

// value of "key": in one entry line (number or string); false if absent
static bool field(const std::string& line, const char* key, std::string* out) {
  const std::string k = std::string("\"") + key + "\"";
  size_t p = line.find(k);
  if (p == std::string::npos) return false;
  p = line.find(':', p + k.size());
  if (p == std::string::npos) return false;
  ++p;
  while (p < line.size() && line[p] == ' ') ++p;
  if (p < line.size() && line[p] == '"') {
    const size_t e = line.find('"', p + 1);
    if (e == std::string::npos) return false;
    *out = line.substr(p + 1, e - p - 1);
    return true;
  }
  size_t e = p;
  while (e < line.size() && (isdigit((unsigned char)line[e]) || line[e] == '.' || line[e] == '-' || line[e] == 'e' ||
                             line[e] == 'E' || line[e] == '+'))
    ++e;
  if (e == p) return false;
  *out = line.substr(p, e - p);
  return true;
}

// Reads the entries of `path` (the caller holds g_tuned_mu).  A missing file
// holds no entries; a line that is not a whole entry is skipped.
static void read_file(const std::string& path) {
  FILE* f = fopen(path.c_str(), "r");
  if (!f) return;
  char buf[1024];
  while (fgets(buf, sizeof buf, f)) {
    const std::string line = buf;
    std::string arch, kind, v[8];
    const char* keys[8] = {"dtype", "bucket", "block", "items", "cutoff", "ms", "default_ms", "version"};
    if (!field(line, "arch", &arch) || !field(line, "kind", &kind)) continue;
    bool ok = true;
    for (int k = 0; k < 7; ++k) ok = ok && field(line, keys[k], &v[k]);
    if (!ok) continue;
    TuneEntry e;
    e.arch = arch;
    e.kind = kind == "batch" ? kTuneBatch : kTuneSingle;
    e.dtype = atoi(v[0].c_str());
    e.bucket = atoi(v[1].c_str());
    e.tn.block = atoi(v[2].c_str());
    e.tn.items = atoi(v[3].c_str());
    e.tn.cutoff = atoi(v[4].c_str());
    e.ms = atof(v[5].c_str());
    e.default_ms = atof(v[6].c_str());
    auto it = std::find_if(g_entries.begin(), g_entries.end(), [&](const TuneEntry& x) {
      return x.arch == e.arch && x.kind == e.kind && x.dtype == e.dtype && x.bucket == e.bucket;
    });
    if (it != g_entries.end())
      *it = e;
    else
      g_entries.push_back(e);
  }
  fclose(f);
}

// Rewrites the file with every known entry (the caller holds g_tuned_mu).
static int write_file() {
  if (g_tune_path.empty()) return KSORT_OK;
  const std::string tmp = g_tune_path + ".tmp";
  FILE* f = fopen(tmp.c_str(), "w");
  if (!f) return fail(KSORT_EINVAL, "cannot write the tuning file " + g_tune_path);
  fprintf(f, "{\"version\": 1, \"entries\": [\n");
  for (size_t k = 0; k < g_entries.size(); ++k) {
    const TuneEntry& e = g_entries[k];
    fprintf(f,
            "{\"arch\": \"%s\", \"kind\": \"%s\", \"dtype\": %d, \"bucket\": %d, \"block\": %d, \"items\": %d, "
            "\"cutoff\": %d, \"ms\": %.6f, \"default_ms\": %.6f}%s\n",
            e.arch.c_str(), kind_name(e.kind), e.dtype, e.bucket, e.tn.block, e.tn.items, e.tn.cutoff, e.ms,
            e.default_ms, k + 1 < g_entries.size() ? "," : "");
  }
  fprintf(f, "]}\n");
  const bool ok = fclose(f) == 0;
  if (!ok || rename(tmp.c_str(), g_tune_path.c_str()) != 0)
    return fail(KSORT_EINVAL, "cannot write the tuning file " + g_tune_path);
  return KSORT_OK;
}

static void check_env_locked() {
  if (g_env_checked) return;
  g_env_checked = true;
  const char* p = getenv("KSORT_TUNE_FILE");
  if (p && *p && g_tune_path.empty()) {
    g_tune_path = p;
    read_file(g_tune_path);
  }
}

bool tuned_for(int dtype, int64_t n, int kind, ksort_tuning* out) {
  static thread_local std::string arch;  // the device of the calling thread, looked up once
  std::lock_guard<std::mutex> lk(g_tuned_mu);
  check_env_locked();
  if (g_entries.empty()) return false;
  if (arch.empty()) arch = device_arch();
  const int b = bucket_of(n);
  for (int d = 0; d <= 2; ++d) {
    for (int sgn : {1, -1}) {
      for (const TuneEntry& e : g_entries) {
        if (e.arch == arch && e.kind == kind && e.dtype == dtype && e.bucket == b + sgn * d) {
          *out = e.tn;
          return true;
        }
      }
      if (d == 0) break;
    }
  }
  return false;
}

// Times variant tn on a copy of src (n keys, packed arrays per d_offsets or
// one array), best of `reps` after a warm-up.
static int time_variant(int dtype, const ksort_tuning& tn, const void* src, void* work, int64_t n,
                        const int64_t* d_offsets, int64_t nseg, size_t kb, hipStream_t st, int reps, double* best_ms) {
  hipEvent_t e0, e1;
  KSORT_HIP(hipEventCreate(&e0));
  KSORT_HIP(hipEventCreate(&e1));
  double best = 1e30;
  int rc = KSORT_OK;
  for (int r = 0; r < reps + 1 && rc == KSORT_OK; ++r) {
    KSORT_HIP(hipMemcpyAsync(work, src, (size_t)n * kb, hipMemcpyDeviceToDevice, st));
    KSORT_HIP(hipEventRecord(e0, st));
    rc = run_sort(dtype, work, n, d_offsets, d_offsets ? nseg : 1, nullptr, &tn, st, d_offsets != nullptr);
    if (rc) break;
    KSORT_HIP(hipEventRecord(e1, st));
    KSORT_HIP(hipEventSynchronize(e1));
    float ms = 0.f;
    KSORT_HIP(hipEventElapsedTime(&ms, e0, e1));
    if (r > 0) best = std::min(best, (double)ms);  // the first run warms up (and records a graph)
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *best_ms = best;
  return rc;
}

// Times every variant of dtype on src and records the fastest for (kind, n).
static int tune_on(int dtype, int kind, const void* src, int64_t n, const int64_t* d_offsets, int64_t nseg,
                   ksort_tuning* out, hipStream_t st) {
  const size_t kb = dtype == KSORT_F64 ? 8 : 4;
  void* work = nullptr;
  KSORT_HIP(hipMalloc(&work, std::max<size_t>((size_t)n * kb, 16)));
  // the variant an untuned call of this kind and size takes
  const Variant* dv = find_variant(dtype, nullptr, n, kind, false);
  const ksort_tuning dflt{dv->block, dv->items, dv->cutoff, 0};
  int rc = KSORT_OK;
  ksort_tuning best{};
  double best_ms = 1e30, default_ms = 0;
  for (const auto& v : variants()) {
    if (v.dtype != dtype) continue;
    ksort_tuning tn{v.block, v.items, v.cutoff, 0};
    double ms = 0;
    rc = time_variant(dtype, tn, src, work, n, d_offsets, nseg, kb, st, 5, &ms);
    if (rc) break;
    if (tn.block == dflt.block && tn.items == dflt.items && tn.cutoff == dflt.cutoff) default_ms = ms;
    if (ms < best_ms) {
      best_ms = ms;
      best = tn;
    }
  }
  (void)hipStreamSynchronize(st);
  (void)hipFree(work);
  if (rc) return rc;
  // another variant replaces the default only when it is at least 1 %
  // faster: closer times are within the spread of repeated runs
  if (default_ms > 0 && best_ms > 0.99 * default_ms) {
    best = dflt;
    best_ms = default_ms;
  }
  {
    std::lock_guard<std::mutex> lk(g_tuned_mu);
    TuneEntry e;
    e.arch = device_arch();
    e.kind = kind;
    e.dtype = dtype;
    e.bucket = bucket_of(n);
    e.tn = best;
    e.ms = best_ms;
    e.default_ms = default_ms;
    auto it = std::find_if(g_entries.begin(), g_entries.end(), [&](const TuneEntry& x) {
      return x.arch == e.arch && x.kind == e.kind && x.dtype == e.dtype && x.bucket == e.bucket;
    });
    if (it != g_entries.end())
      *it = e;
    else
      g_entries.push_back(e);
    rc = write_file();
  }
  if (out) *out = best;
  return rc;
}

}  // namespace ksort

using namespace ksort;

extern "C" {

int ksort_autotune(int dtype, int64_t n, ksort_tuning* out, void* stream) {
  if (dtype != KSORT_F64 && dtype != KSORT_F32) return fail(KSORT_EINVAL, "bad dtype");
  if (n < 2 || n > ((int64_t)1 << 31) - 1) return fail(KSORT_EINVAL, "autotune needs 2 <= n < 2^31");
  const size_t kb = dtype == KSORT_F64 ? 8 : 4;
  hipStream_t st = (hipStream_t)stream;
  void* src = nullptr;
  KSORT_HIP(hipMalloc(&src, (size_t)n * kb));
  if (dtype == KSORT_F64)
    hipLaunchKernelGGL(fill_uniform<double>, dim3(1024), dim3(256), 0, st, (double*)src, n, 0x5EEDull);
  else
    hipLaunchKernelGGL(fill_uniform<float>, dim3(1024), dim3(256), 0, st, (float*)src, n, 0x5EEDull);
  const int rc = tune_on(dtype, kTuneSingle, src, n, nullptr, 1, out, st);
  (void)hipStreamSynchronize(st);
  (void)hipFree(src);
  return rc;
}

int ksort_autotune_batch(int dtype, const void* d_packed, int64_t n_total, const int64_t* d_offsets, int64_t nseg,
                         ksort_tuning* out, void* stream) {
  if (dtype != KSORT_F64 && dtype != KSORT_F32) return fail(KSORT_EINVAL, "bad dtype");
  if (n_total < 2 || n_total > ((int64_t)1 << 31) - 1 || nseg < 1)
    return fail(KSORT_EINVAL, "autotune needs 2 <= n_total < 2^31 and nseg >= 1");
  if (!d_packed || !d_offsets) return fail(KSORT_EINVAL, "null pointer");
  return tune_on(dtype, kTuneBatch, d_packed, n_total, d_offsets, nseg, out, (hipStream_t)stream);
}

int ksort_tune_file(const char* path) {
  std::lock_guard<std::mutex> lk(g_tuned_mu);
  g_env_checked = true;  // an explicit file replaces KSORT_TUNE_FILE
  if (!path) {
    // forget every choice: calls take the untuned defaults again
    g_tune_path.clear();
    g_entries.clear();
    return KSORT_OK;
  }
  g_tune_path = path;
  read_file(g_tune_path);
  return KSORT_OK;
}

int ksort_tune_count(void) {
  std::lock_guard<std::mutex> lk(g_tuned_mu);
  check_env_locked();
  return (int)g_entries.size();
}

}  // extern "C"
