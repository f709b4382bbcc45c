// K-sort library for MI355X (gfx950): host level driver and C ABI.
//
// A sort runs as a sequence of stage launches.  Stage 0 holds the input
// arrays; stage s partitions every live segment once (Steps 1-4 of
// arXiv 1107.3622, Section 1.1) and finishes in LDS every segment of at most
// `cutoff` keys that stage s-1 produced; its two sides (Steps 5-6) become the
// segments of stage s+1.  The device keeps all lists and counters, so the host
// only launches stages in batches and reads one flag word after each batch to
// learn whether work is left.
#include <dlfcn.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "ksort.h"
#include "ksort_engine.h"
#include "ksort_epoch.h"
#include "ksort_kernels.h"

namespace ksort {

// ---------------------------------------------------------------- errors

static thread_local std::string t_last_error;

void set_error(const std::string& msg) { t_last_error = msg; }

int fail(int code, const std::string& msg) {
  set_error(msg);
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  char buf[512];
  snprintf(buf, sizeof buf, "%s failed: %s (%d)", what, hipGetErrorString(e), (int)e);
  set_error(buf);
  return e == hipErrorOutOfMemory ? KSORT_ENOMEM : KSORT_EHIP;
}

// ---------------------------------------------------------------- variants

template <typename T, int BLOCK, int ITEMS, int CUT>
static Variant make_variant(int dtype) {
  Variant v;
  v.dtype = dtype;
  v.block = BLOCK;
  v.items = ITEMS;
  v.cutoff = CUT;
  v.stage = (const void*)&stage_kernel<T, BLOCK, ITEMS, CUT>;
  v.launch = [](const StageArgs& a, int grid, hipStream_t stream) -> hipError_t {
    hipLaunchKernelGGL((stage_kernel<T, BLOCK, ITEMS, CUT>), dim3(grid), dim3(BLOCK), 0, stream, a);
    return hipGetLastError();
  };
  v.key_bytes = sizeof(T);
  return v;
}

const std::vector<Variant>& variants() {
  static const std::vector<Variant> vs = {
      make_variant<double, 512, 24, 2048>(KSORT_F64),
      make_variant<double, 512, 28, 2048>(KSORT_F64),
      make_variant<double, 512, 16, 2048>(KSORT_F64),
      make_variant<double, 1024, 8, 2048>(KSORT_F64),
      make_variant<double, 512, 16, 1024>(KSORT_F64),
      make_variant<double, 256, 24, 2048>(KSORT_F64),
      make_variant<double, 256, 32, 2048>(KSORT_F64),
      make_variant<float, 512, 32, 2048>(KSORT_F32),
      make_variant<float, 512, 24, 2048>(KSORT_F32),
      make_variant<float, 512, 16, 2048>(KSORT_F32),
      make_variant<float, 1024, 8, 2048>(KSORT_F32),
      make_variant<float, 512, 16, 1024>(KSORT_F32),
      make_variant<float, 256, 32, 2048>(KSORT_F32),
  };
  return vs;
}

static std::mutex g_default_mu;
static int g_default[2] = {-1, -1};

static int variant_index(int dtype, int block, int items, int cutoff) {
  const auto& vs = variants();
  for (size_t j = 0; j < vs.size(); ++j)
    if (vs[j].dtype == dtype && vs[j].block == block && vs[j].items == items && vs[j].cutoff == cutoff)
      return (int)j;
  return -1;
}

static constexpr int64_t kSmallSortKeys = 3000000;

const Variant* find_variant(int dtype, const ksort_tuning* tune, int64_t n, int kind, bool use_tuned) {
  if (dtype != KSORT_F64 && dtype != KSORT_F32) return nullptr;
  const auto& vs = variants();
  if (tune && (tune->block || tune->items || tune->cutoff)) {
    const int j = variant_index(dtype, tune->block, tune->items, tune->cutoff);
    return j < 0 ? nullptr : &vs[j];
  }
  ksort_tuning tn;
  if (use_tuned && n >= 0 && tuned_for(dtype, n, kind, &tn)) {
    const int j = variant_index(dtype, tn.block, tn.items, tn.cutoff);
    if (j >= 0) return &vs[j];
  }
  std::lock_guard<std::mutex> lk(g_default_mu);
  int j = g_default[dtype];
  // Arrays below 3e6 keys (measured crossover between 2.5e6 and 4e6) sort
  // faster with 16 keys per thread and a 1024-key LDS finish: more, shorter
  // finish tasks at the levels that dominate small sorts (1e5: 0.29 against
  // 0.32 ms, 1e6: 0.51 against 0.57, 2.5e6: 0.70 against 0.72; 4e6: 0.89
  // against 0.84).  A default set by the caller or a tuned bucket wins.
  if (j < 0 && n >= 0 && n < kSmallSortKeys) j = variant_index(dtype, 512, 16, 1024);
  // FP32 keys take 32 per thread: a tile then moves 64 KB, near the 96 KB
  // of an FP64 tile of 24, which keeps the per-tile scan and look-back cost
  // small against the data moved on large arrays
  if (j < 0) j = dtype == KSORT_F64 ? variant_index(dtype, 512, 24, 2048) : variant_index(dtype, 512, 32, 2048);
  // FP64 arrays whose full passes need a second round of 12288-key tiles on
  // the 512-workgroup grid of a 256-CU device but fit one round of
  // 14336-key tiles: 28 keys per thread (7e6 keys: 0.993 against 1.010 ms)
  if (g_default[dtype] < 0 && dtype == KSORT_F64 && n > 512LL * 512 * 24 && n <= 512LL * 512 * 28)
    j = variant_index(dtype, 512, 28, 2048);
  return &vs[j];
}

int set_default_variant(int dtype, const ksort_tuning* tune) {
  if (dtype != KSORT_F64 && dtype != KSORT_F32) return fail(KSORT_EINVAL, "bad dtype");
  int j = -1;
  if (tune) {
    j = variant_index(dtype, tune->block, tune->items, tune->cutoff);
    if (j < 0) return fail(KSORT_EINVAL, "no such kernel variant");
  }
  std::lock_guard<std::mutex> lk(g_default_mu);
  g_default[dtype] = j;
  return KSORT_OK;
}

// ---------------------------------------------------------------- device info

static std::mutex g_dev_mu;
static std::map<int, std::unique_ptr<DeviceInfo>> g_devs;

int device_info(int ordinal, const DeviceInfo** out) {
  std::lock_guard<std::mutex> lk(g_dev_mu);
  auto it = g_devs.find(ordinal);
  if (it != g_devs.end()) {
    *out = it->second.get();
    return KSORT_OK;
  }
  hipDeviceProp_t prop;
  KSORT_HIP(hipGetDeviceProperties(&prop, ordinal));
  auto di = std::make_unique<DeviceInfo>();
  di->ordinal = ordinal;
  di->cus = prop.multiProcessorCount;
  di->arch = prop.gcnArchName;
  di->gfx950 = di->arch.rfind("gfx950", 0) == 0;
  for (const auto& v : variants()) {
    int nb = 0;
    KSORT_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, v.stage, v.block, 0));
    di->occupancy.push_back(std::max(nb, 1));
  }
  *out = di.get();
  g_devs[ordinal] = std::move(di);
  return KSORT_OK;
}

// ---------------------------------------------------------------- capacities

Caps caps_for(const Variant& v, int64_t n, int64_t nseg, bool level_mode) {
  Caps c;
  if (level_mode) {
    c.live = nseg + 2;
    c.tiles = n / v.tile() + nseg + 2;
    c.fin = 2;
  } else {
    // live segments have more than `cutoff` keys and are disjoint
    c.live = n / (v.cutoff + 1) + 2;
    c.tiles = n / v.tile() + c.live + 2;
    // stage 0 may hold every small input array; later stages at most
    // kChainLists sides per live segment of the stage before (two, or more
    // when a chain of one-tile segments is partitioned within the pass)
    c.fin = std::max<int64_t>(nseg, (int64_t)kChainLists * c.live) + 2;
    // a sort of n keys takes at most about n level passes (ordered inputs)
    c.stats = std::min<int64_t>(n, 65536) + 64;
  }
  return c;
}

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

static size_t arena_bytes_for(const Caps& c, int cap_stats) {
  size_t b = 0;
  b += align256(3 * sizeof(StageCtr));
  b += align256(sizeof(Flags));
  b += 2 * align256((size_t)c.live * sizeof(Seg));
  b += 2 * align256((size_t)c.tiles * sizeof(int32_t));
  b += 2 * align256((size_t)2 * c.fin * sizeof(Seg));  // children below caps.fin, carried tasks above
  b += align256((size_t)c.tiles * sizeof(uint64_t));
  b += align256((size_t)cap_stats * 2 * sizeof(int64_t));
  b += 2 * align256((size_t)c.bufs * sizeof(int32_t));
  return b;
}

Workspace::~Workspace() {
  for (auto e : events) (void)hipEventDestroy(e);
  if (capture) (void)hipStreamDestroy(capture);
  if (!user) {
    if (arena) (void)hipFree(arena);
    if (scratch) (void)hipFree(scratch);
  }
  if (h_flags && own_h_flags) (void)hipHostFree(h_flags);
}

// Lays out the descriptor lists, counters, flags and look-back words in
// `base` for caps `nc` and clears them.
static int carve_arena(Workspace& w, void* base, const Caps& nc, size_t bytes) {
  w.arena = base;
  w.arena_bytes = bytes;
  w.caps = nc;
  w.cap_stats = (int)nc.stats;
  char* p = (char*)base;
  auto take = [&](size_t sz) {
    char* r = p;
    p += align256(sz);
    return (void*)r;
  };
  w.ctr = (StageCtr*)take(3 * sizeof(StageCtr));
  w.flags = (Flags*)take(sizeof(Flags));
  for (int k = 0; k < 2; ++k) w.live[k] = (Seg*)take((size_t)nc.live * sizeof(Seg));
  for (int k = 0; k < 2; ++k) w.tilemap[k] = (int32_t*)take((size_t)nc.tiles * sizeof(int32_t));
  for (int k = 0; k < 2; ++k) w.fin[k] = (Seg*)take((size_t)2 * nc.fin * sizeof(Seg));
  w.status = (uint64_t*)take((size_t)nc.tiles * sizeof(uint64_t));
  w.stage_keys = (int64_t*)take((size_t)w.cap_stats * 2 * sizeof(int64_t));
  w.pending = (int32_t*)take((size_t)nc.bufs * sizeof(int32_t));
  w.done_stage = (int32_t*)take((size_t)nc.bufs * sizeof(int32_t));
  KSORT_HIP(hipMemsetAsync(base, 0, bytes, w.stream));
  w.epoch = 0;
  ++w.generation;
  return KSORT_OK;
}

int Workspace::reserve(const Caps& c, size_t scratch_need) {
  if (!h_flags) KSORT_HIP(hipHostMalloc((void**)&h_flags, sizeof(Flags), hipHostMallocDefault));
  const bool fits = arena && c.live <= caps.live && c.tiles <= caps.tiles && c.fin <= caps.fin &&
                    c.bufs <= caps.bufs && c.stats <= caps.stats;
  Caps nc = caps;
  if (!fits) {
    nc.live = std::max(c.live, caps.live);
    nc.tiles = std::max(c.tiles, caps.tiles);
    nc.fin = std::max(c.fin, caps.fin);
    nc.bufs = std::max(c.bufs, caps.bufs);
    nc.stats = std::max(c.stats, caps.stats);
  }
  if (user) {
    // the caller's memory: arena first, the scratch after it; nothing is
    // allocated, a call that needs more fails
    const size_t ab = arena_bytes_for(nc, (int)nc.stats);
    const size_t need = align256(ab) + align256(std::max<size_t>(scratch_need, 1));
    if (need > user_bytes)
      return fail(KSORT_ENOMEM, "the workspace given to ksort_set_workspace holds " + std::to_string(user_bytes) +
                                    " bytes; this call needs " + std::to_string(need));
    if (!fits) {
      int rc = carve_arena(*this, user, nc, ab);
      if (rc) return rc;
    }
    char* const sc = (char*)user + align256(arena_bytes);
    if (sc != scratch) ++generation;
    scratch = sc;
    scratch_bytes = user_bytes - align256(arena_bytes);
    return KSORT_OK;
  }
  if (!fits) {
    if (arena) {
      KSORT_HIP(hipStreamSynchronize(stream));
      KSORT_HIP(hipFree(arena));
      arena = nullptr;
    }
    const size_t bytes = arena_bytes_for(nc, (int)nc.stats);
    void* base = nullptr;
    KSORT_HIP(hipMalloc(&base, bytes));
    int rc = carve_arena(*this, base, nc, bytes);
    if (rc) return rc;
  }
  if (scratch_need > scratch_bytes) {
    if (scratch) {
      KSORT_HIP(hipStreamSynchronize(stream));
      KSORT_HIP(hipFree(scratch));
      scratch = nullptr;
      scratch_bytes = 0;
    }
    KSORT_HIP(hipMalloc(&scratch, scratch_need));
    scratch_bytes = scratch_need;
    ++generation;
  }
  return KSORT_OK;
}

int Workspace::use_memory(void* d, size_t bytes) {
  KSORT_HIP(hipStreamSynchronize(stream));
  if (!user) {
    if (arena) KSORT_HIP(hipFree(arena));
    if (scratch) KSORT_HIP(hipFree(scratch));
  }
  arena = nullptr;
  scratch = nullptr;
  arena_bytes = scratch_bytes = 0;
  caps = Caps{};
  ++generation;
  user = d;
  user_bytes = d ? bytes : 0;
  return KSORT_OK;
}

static std::mutex g_ws_mu;
static std::map<std::pair<int, hipStream_t>, std::unique_ptr<Workspace>> g_ws;

Workspace* workspace_for(int device, hipStream_t stream) {
  std::lock_guard<std::mutex> lk(g_ws_mu);
  auto key = std::make_pair(device, stream);
  auto it = g_ws.find(key);
  if (it != g_ws.end()) return it->second.get();
  auto ws = std::make_unique<Workspace>();
  ws->device = device;
  ws->stream = stream;
  Workspace* r = ws.get();
  g_ws[key] = std::move(ws);
  return r;
}

void release_workspaces() {
  std::lock_guard<std::mutex> lk(g_ws_mu);
  g_ws.clear();
}

// ---------------------------------------------------------------- launches

#ifndef KSORT_FIN_RUN
#define KSORT_FIN_RUN(grid) (grid)
#endif


// Polls a look-back wait makes before its pass gives up with an error.  A
// tile waits only for tiles that running workgroups hold, which publish within
// microseconds; 2^22 polls take seconds.  KSORT_SPIN_LIMIT (a decimal count)
// overrides it, read whenever a pass is enqueued (a captured graph keeps the
// value it was captured with); tests use a tiny limit to force the error.
// Whether the library's own passes give workgroup b ticket b without the
// counter (KSORT_FIXED_FIRST=0 takes every ticket from the counter).
static int fixed_first_setting() {
  const char* s = getenv("KSORT_FIXED_FIRST");
  return s && s[0] == '0' && s[1] == '\0' ? 0 : 1;
}

uint32_t spin_limit_setting() {
  constexpr uint32_t kDefault = 1u << 22;
  const char* s = getenv("KSORT_SPIN_LIMIT");
  if (!s || !*s) return kDefault;
  char* end = nullptr;
  const unsigned long long v = strtoull(s, &end, 10);
  if (*end != '\0' || v > 0xffffffffull) return kDefault;
  return (uint32_t)v;
}

StageArgs stage_args(Workspace& ws, const Variant& v, int stage, int64_t* pivot_out, int pivot_relative,
                     int emit_children) {
  StageArgs a;
  memset(&a, 0, sizeof a);
  a.ctr = ws.ctr;
  for (int k = 0; k < 2; ++k) {
    a.live[k] = ws.live[k];
    a.tilemap[k] = ws.tilemap[k];
    a.fin[k] = ws.fin[k];
  }
  a.status = ws.status;
  a.pivot_out = pivot_out;
  a.pending = nullptr;
  a.done_stage = nullptr;
  a.flags = ws.flags;
  a.stage_keys = ws.stats ? ws.stage_keys : nullptr;  // counted only for profiling
  a.cap_live = (int32_t)ws.caps.live;
  a.cap_tiles = (int32_t)ws.caps.tiles;
  // A stage's finish list holds the children of the stage before below
  // caps.fin and the finish tasks carried over from it above.
  a.fin_half = (int32_t)ws.caps.fin;
  a.cap_fin = (int32_t)(2 * ws.caps.fin);
  a.fin_run = 0;  // launch_stage: one round of the grid
  a.cap_stats = ws.cap_stats;
  a.stage = stage;
  a.epoch = epoch_of(stage, ws.epoch_span);
  a.cutoff = v.cutoff;
  a.emit_children = emit_children;
  a.pivot_relative = pivot_relative;
  a.spin_limit = spin_limit_setting();
  a.fixed_first = fixed_first_setting();
  return a;
}

int flags_error(const Flags& f) {
  if (f.overflow == 4) {
    char buf[256];
    snprintf(buf, sizeof buf,
             "a look-back wait timed out (pass %d: tile %d waited for tile %d, whose word was 0x%016llx)",
             f.diag_stage, f.diag_tile, f.diag_pred, (unsigned long long)f.diag_word);
    return fail(KSORT_EINTERNAL, buf);
  }
  if (f.overflow) return fail(KSORT_EINTERNAL, "device consistency check failed (code " + std::to_string(f.overflow) + ")");
  return KSORT_OK;
}

// ---------------------------------------------------------------- launch order

struct OrderedLaunches::Order {
  std::mutex mu;
  hipEvent_t last = nullptr;  // end of the latest batch of stage launches on the device
};

static std::mutex g_order_mu;
static std::map<int, std::unique_ptr<OrderedLaunches::Order>> g_order;

OrderedLaunches::OrderedLaunches(int device, hipStream_t stream) : stream_(stream) {
  {
    std::lock_guard<std::mutex> lk(g_order_mu);
    auto& p = g_order[device];
    if (!p) p.reset(new Order);
    o_ = p.get();
  }
  o_->mu.lock();
  hipError_t e = hipSuccess;
  if (!o_->last)
    e = hipEventCreateWithFlags(&o_->last, hipEventDisableTiming);
  else
    e = hipStreamWaitEvent(stream, o_->last, 0);
  if (e != hipSuccess) rc_ = hip_fail(e, "ordering stage launches");
}

OrderedLaunches::~OrderedLaunches() {
  if (o_->last) (void)hipEventRecord(o_->last, stream_);
  o_->mu.unlock();
}

int launch_reset(Workspace& ws) {
  const int64_t nwords = ws.caps.tiles;
  const int blocks = (int)std::min<int64_t>(1024, (nwords + 255) / 256);
  if (ws.stats) {
    const int64_t nk = 2 * (int64_t)ws.cap_stats;
    hipLaunchKernelGGL(clear_kernel, dim3((unsigned)std::min<int64_t>(256, (nk + 255) / 256)), dim3(256), 0, ws.stream,
                       (uint64_t*)ws.stage_keys, nk);
    KSORT_HIP(hipGetLastError());
  }
  hipLaunchKernelGGL(reset_kernel, dim3(std::max(blocks, 1)), dim3(256), 0, ws.stream, ws.ctr, ws.flags, ws.status,
                     nwords);
  KSORT_HIP(hipGetLastError());
  return KSORT_OK;
}

int launch_clear_status(Workspace& ws) {
  const int64_t nwords = ws.caps.tiles;
  const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>(1024, (nwords + 255) / 256));
  hipLaunchKernelGGL(clear_kernel, dim3(blocks), dim3(256), 0, ws.stream, ws.status, nwords);
  KSORT_HIP(hipGetLastError());
  return KSORT_OK;
}

int launch_init(Workspace& ws, const Variant& v, const InitArgs& ia, int64_t nblocks) {
  (void)v;
  if (nblocks <= 0) return KSORT_OK;
  if (nblocks > 0x7fffffff) return fail(KSORT_EINVAL, "too many arrays");
  hipLaunchKernelGGL(init_kernel, dim3((uint32_t)nblocks), dim3(256), 0, ws.stream, ia);
  KSORT_HIP(hipGetLastError());
  return KSORT_OK;
}

int stage_grid(const Variant& v, const DeviceInfo& di, const Caps& c) {
  const auto& vs = variants();
  const int idx = (int)(&v - vs.data());
  const int64_t full = (int64_t)di.occupancy[idx] * di.cus;
  const int64_t work = c.tiles + c.fin;
  return (int)std::max<int64_t>(1, std::min(full, work));
}

int launch_stage(Workspace& ws, const Variant& v, const StageArgs& a, int grid) {
  StageArgs args = a;
  // unless the caller chose otherwise, one round of finish tasks on the grid
  // in a stage that also partitions
  if (args.fin_run <= 0) args.fin_run = KSORT_FIN_RUN(grid);
  KSORT_HIP(v.launch(args, grid, ws.stream));
  return KSORT_OK;
}

// Segments become one tile after about 2.6 log2(n / tile) levels on random
// keys; from there a chain of one-tile segments runs within one pass and the
// finish takes one more (measured: 12, 21 and 28 passes with work at 1e5, 1e6
// and 7e6 keys).  Two spare passes cover most seeds; a short batch costs one
// more round trip, an idle pass about 6 us.
int predict_stages(int64_t n, int cutoff, int tile) {
  if (n <= cutoff) return 1;
  if (n <= tile) return 4;
  const double r = std::log2((double)n / (double)tile);
  return (int)std::ceil(2.6 * r) + 6;
}

// ---------------------------------------------------------------- profiling

static std::atomic<int> g_profile{0};
static std::mutex g_prof_mu;
static std::vector<ksort_level_record> g_prof;
static std::atomic<int64_t> g_call{0};

// KSORT_TRACE=<path>: every sorting call runs with per-pass events and
// appends one JSON line per level pass to <path> (read once, at first use).
static const std::string& trace_path() {
  static const std::string p = [] {
    const char* e = getenv("KSORT_TRACE");
    return std::string(e ? e : "");
  }();
  return p;
}

bool profiling_on() { return g_profile.load() != 0; }
static bool tracing_on() { return !trace_path().empty(); }
void profile_push(const ksort_level_record& r) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  if (profiling_on()) g_prof.push_back(r);
  if (tracing_on()) {
    static FILE* f = fopen(trace_path().c_str(), "a");
    if (f) {
      fprintf(f,
              "{\"call\": %lld, \"dtype\": \"%s\", \"stage\": %d, \"live_keys\": %lld, \"finish_keys\": %lld, "
              "\"ms\": %.6f, \"block\": %d, \"items\": %d, \"cutoff\": %d, \"grid\": %d}\n",
              (long long)r.call, r.dtype == KSORT_F64 ? "f64" : "f32", r.stage, (long long)r.live_keys,
              (long long)r.finish_keys, r.ms, r.block, r.items, r.cutoff, r.grid);
      fflush(f);
    }
  }
}

// KSORT_ROCTX=1: a roctx range around every batch of level passes, for
// profilers that show host-side markers (rocprofv3 --marker-trace).  The
// roctx library is loaded at first use, if it is there.
struct Roctx {
  int (*push)(const char*) = nullptr;
  int (*pop)() = nullptr;
};
static const Roctx& roctx() {
  static const Roctx r = [] {
    Roctx x;
    const char* e = getenv("KSORT_ROCTX");
    if (!e || strcmp(e, "1") != 0) return x;
    void* h = dlopen("librocprofiler-sdk-roctx.so.1", RTLD_NOW | RTLD_LOCAL);
    if (!h) h = dlopen("libroctx64.so.4", RTLD_NOW | RTLD_LOCAL);
    if (!h) return x;
    x.push = (int (*)(const char*))dlsym(h, "roctxRangePushA");
    x.pop = (int (*)())dlsym(h, "roctxRangePop");
    if (!x.push || !x.pop) x = Roctx{};
    return x;
  }();
  return r;
}

struct RoctxRange {
  bool on;
  RoctxRange(int stage0, int stages, int64_t n) : on(roctx().push != nullptr) {
    if (!on) return;
    char buf[96];
    snprintf(buf, sizeof buf, "ksort passes %d..%d (n=%lld)", stage0, stage0 + stages - 1, (long long)n);
    roctx().push(buf);
  }
  ~RoctxRange() {
    if (on) roctx().pop();
  }
};
int64_t next_call_id() { return g_call.fetch_add(1); }

// ---------------------------------------------------------------- graphs

struct GraphKey {
  int dtype;
  void* data;
  int64_t n;
  const int64_t* offsets;
  int64_t nseg;
  int64_t* pivots;
  const Variant* v;
  bool operator<(const GraphKey& o) const {
    return std::tie(dtype, data, n, offsets, nseg, pivots, v) <
           std::tie(o.dtype, o.data, o.n, o.offsets, o.nseg, o.pivots, o.v);
  }
};

struct GraphEntry {
  hipGraphExec_t exec = nullptr;
  int stages = 0;
  uint64_t generation = 0;  // layout of the workspace the graph was recorded with
  int64_t epoch_span = 0;   // look-back tag span its passes used
  uint64_t last_use = 0;
};

// Recorded graphs are kept per (workspace, arguments), at most kMaxGraphs of
// them; the least recently used one is dropped first.  A graph holds the
// pointers and list capacities of the workspace layout it was recorded
// with, so it is used only while that layout (its generation) is current.
constexpr size_t kMaxGraphs = 64;
static std::mutex g_graph_mu;
static std::map<std::pair<Workspace*, GraphKey>, GraphEntry> g_graphs;
static uint64_t g_graph_clock = 0;

static void evict_lru_graph() {
  auto victim = g_graphs.end();
  for (auto it = g_graphs.begin(); it != g_graphs.end(); ++it)
    if (victim == g_graphs.end() || it->second.last_use < victim->second.last_use) victim = it;
  if (victim != g_graphs.end()) {
    (void)hipGraphExecDestroy(victim->second.exec);
    g_graphs.erase(victim);
  }
}

// ---------------------------------------------------------------- the sort

static int enqueue_prologue(Workspace& ws, const Variant& v, int dtype, void* d_data, int64_t n,
                            const int64_t* d_offsets, int64_t nseg, int64_t* d_pivots) {
  (void)dtype;
  int rc = launch_reset(ws);
  if (rc) return rc;
  InitArgs ia;
  memset(&ia, 0, sizeof ia);
  ia.sa = stage_args(ws, v, 0, d_pivots, 1, 1);
  ia.pair.data = d_data;
  ia.pair.scratch = ws.scratch;
  ia.buf = 0;
  ia.root_base = 0;
  ia.n = n;
  ia.offsets = d_offsets;
  ia.seg_left = nullptr;
  ia.seg_len = nullptr;
  ia.nseg = nseg;
  ia.level_mode = 0;
  ia.tile = v.tile();
  return launch_init(ws, v, ia, nseg);
}

// Keys in the longest array of a packed batch (offsets read back once): the
// recursion depth, and so the passes to launch, follow the longest array,
// not the total.  Offsets the init kernel would reject count as empty.
static int longest_array(const int64_t* d_offsets, int64_t nseg, int64_t n, hipStream_t stream, int64_t* out) {
  std::vector<int64_t> h((size_t)nseg + 1);
  KSORT_HIP(hipMemcpyAsync(h.data(), d_offsets, h.size() * sizeof(int64_t), hipMemcpyDeviceToHost, stream));
  KSORT_HIP(hipStreamSynchronize(stream));
  int64_t m = 0;
  for (int64_t u = 0; u < nseg; ++u) {
    const int64_t len = h[(size_t)u + 1] - h[(size_t)u];
    if (len > m && len <= n) m = len;
  }
  *out = m;
  return KSORT_OK;
}

static int sort_in(Workspace& ws, const Variant& v, const DeviceInfo& di, int dtype, void* d_data, int64_t n,
                   const int64_t* d_offsets, int64_t nseg, int64_t* d_pivots, hipStream_t stream, bool use_graph,
                   bool allow_profiling);

// ---------------------------------------------------------------- contract check
//
// The sort's output is the unique ascending arrangement, bit for bit, when
// the keys hold no NaN and not both zeros (+0.0 and -0.0 compare equal, so
// their relative order depends on the algorithm).  With KSORT_VALIDATE=1
// the sorting calls check that first and refuse other inputs.

// flags[0]: a NaN, flags[1]: a +0.0, flags[2]: a -0.0 (one atomic per wave
// that found any)
__device__ __forceinline__ bool sign_set(double v) { return __double_as_longlong(v) < 0; }
__device__ __forceinline__ bool sign_set(float v) { return __float_as_int(v) < 0; }

template <typename T>
__global__ void contract_kernel(const T* d, int64_t n, int32_t* flags) {
  bool nan = false, pz = false, nz = false;
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n; x += (int64_t)gridDim.x * blockDim.x) {
    const T v = d[x];
    nan = nan || v != v;
    if (v == T(0)) {
      if (sign_set(v))
        nz = true;
      else
        pz = true;
    }
  }
  const uint64_t bn = __ballot(nan), bp = __ballot(pz), bz = __ballot(nz);
  if ((threadIdx.x & (kWave - 1)) == 0) {
    if (bn) atomicOr(flags, 1);
    if (bp) atomicOr(flags + 1, 1);
    if (bz) atomicOr(flags + 2, 1);
  }
}

static bool validating() {
  const char* e = getenv("KSORT_VALIDATE");
  return e && e[0] == '1' && e[1] == '\0';
}

static int check_contract(int dtype, const void* d, int64_t n, hipStream_t st) {
  if (n <= 0) return KSORT_OK;
  int32_t* dflags = nullptr;  // a debugging aid: one small allocation per call
  KSORT_HIP(hipMalloc((void**)&dflags, 3 * sizeof(int32_t)));
  int32_t h[3] = {0, 0, 0};
  hipError_t e = hipMemsetAsync(dflags, 0, sizeof h, st);
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 2048));
  if (e == hipSuccess) {
    if (dtype == KSORT_F64)
      hipLaunchKernelGGL(contract_kernel<double>, dim3(grid), dim3(256), 0, st, (const double*)d, n, dflags);
    else
      hipLaunchKernelGGL(contract_kernel<float>, dim3(grid), dim3(256), 0, st, (const float*)d, n, dflags);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpyAsync(h, dflags, sizeof h, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  (void)hipFree(dflags);
  if (e != hipSuccess) return hip_fail(e, "contract check");
  if (h[0]) return fail(KSORT_EINVAL, "KSORT_VALIDATE: the keys hold a NaN (outside the bit-exact contract)");
  if (h[1] && h[2]) return fail(KSORT_EINVAL, "KSORT_VALIDATE: the keys hold both +0.0 and -0.0 (outside the bit-exact contract)");
  return KSORT_OK;
}

int run_sort(int dtype, void* d_data, int64_t n, const int64_t* d_offsets, int64_t nseg, int64_t* d_pivots,
             const ksort_tuning* tune, hipStream_t stream, bool use_graph) {
  if (dtype != KSORT_F64 && dtype != KSORT_F32) return fail(KSORT_EINVAL, "bad dtype");
  if (n < 0 || nseg < 0) return fail(KSORT_EINVAL, "negative size");
  if (n > 0 && !d_data) return fail(KSORT_EINVAL, "null data pointer");
  if (d_offsets == nullptr && nseg != 1) return fail(KSORT_EINVAL, "internal: single array needs nseg == 1");
  if (n > ((int64_t)1 << 31) - 1) return fail(KSORT_EINVAL, "more than 2^31-1 keys");
  const Variant* v = find_variant(dtype, tune, n, d_offsets ? kTuneBatch : kTuneSingle);
  if (!v) return fail(KSORT_EINVAL, "no such kernel variant");
  if (nseg == 0) return KSORT_OK;
  if (validating()) {
    const int vrc = check_contract(dtype, d_data, n, stream);
    if (vrc) return vrc;
  }
  if (d_offsets == nullptr && n <= 1) {
    if (d_pivots) {
      const int64_t fp = n == 0 ? -1 : 0;
      KSORT_HIP(hipMemcpyAsync(d_pivots, &fp, sizeof fp, hipMemcpyHostToDevice, stream));
      KSORT_HIP(hipStreamSynchronize(stream));
    }
    return KSORT_OK;
  }
  int dev = 0;
  KSORT_HIP(hipGetDevice(&dev));
  const DeviceInfo* di = nullptr;
  int rc = device_info(dev, &di);
  if (rc) return rc;
  if (!di->gfx950) return fail(KSORT_EUNSUPPORTED, "device " + std::to_string(dev) + " is " + di->arch + ", not gfx950");

  Workspace& ws = *workspace_for(dev, stream);
  std::lock_guard<std::mutex> lk(ws.mu);
  return sort_in(ws, *v, *di, dtype, d_data, n, d_offsets, nseg, d_pivots, stream, use_graph, true);
}

// The level loop of one sort in workspace ws (whose lock the caller holds).
static int sort_in(Workspace& ws, const Variant& vv, const DeviceInfo& dinfo, int dtype, void* d_data, int64_t n,
                   const int64_t* d_offsets, int64_t nseg, int64_t* d_pivots, hipStream_t stream, bool use_graph,
                   bool allow_profiling) {
  const Variant* v = &vv;
  const DeviceInfo* di = &dinfo;
  const int dev = di->ordinal;
  ws.stream = stream;
  const Caps caps = caps_for(*v, n, nseg, false);
  int rc = ws.reserve(caps, (size_t)std::max<int64_t>(n, 1) * v->key_bytes);
  if (rc) return rc;
  const int grid = stage_grid(*v, *di, ws.caps);
  const bool prof = allow_profiling && (profiling_on() || tracing_on());
  ws.stats = prof;
  ws.epoch_span = epoch_span_setting();
  const int64_t call = next_call_id();

  int stage = 0;
  int batch = predict_stages(n, v->cutoff, v->tile());
  int more = 4;  // the batch after a short one; doubles up to 64
  bool graphed = false;

  if (use_graph && !prof) {
    GraphKey key{dtype, d_data, n, d_offsets, nseg, d_pivots, v};
    std::lock_guard<std::mutex> gl(g_graph_mu);
    auto gk = std::make_pair(&ws, key);
    auto it = g_graphs.find(gk);
    if (it != g_graphs.end() && it->second.generation != ws.generation) {
      (void)hipGraphExecDestroy(it->second.exec);
      g_graphs.erase(it);
      it = g_graphs.end();
    }
    if (it == g_graphs.end()) {
      while (g_graphs.size() >= kMaxGraphs) evict_lru_graph();
      if (d_offsets) {
        int64_t longest = n;
        if ((rc = longest_array(d_offsets, nseg, n, stream, &longest))) return rc;
        batch = predict_stages(longest, v->cutoff, v->tile());
      }
      // Record on a private stream (the caller's may be the legacy null
      // stream, which cannot be captured); the graph is launched on the
      // caller's stream.
      if (!ws.capture) KSORT_HIP(hipStreamCreateWithFlags(&ws.capture, hipStreamNonBlocking));
      hipGraph_t g = nullptr;
      KSORT_HIP(hipStreamBeginCapture(ws.capture, hipStreamCaptureModeThreadLocal));
      const hipStream_t user = ws.stream;
      ws.stream = ws.capture;
      int crc = enqueue_prologue(ws, *v, dtype, d_data, n, d_offsets, nseg, d_pivots);
      for (int s = 0; s < batch && crc == KSORT_OK; ++s) {
        if (epoch_wraps_before(s, ws.epoch_span)) crc = launch_clear_status(ws);
        if (crc == KSORT_OK) crc = launch_stage(ws, *v, stage_args(ws, *v, s, d_pivots, 1, 1), grid);
      }
      if (crc == KSORT_OK) {
        hipError_t e = hipMemcpyAsync(ws.h_flags, ws.flags, sizeof(Flags), hipMemcpyDeviceToHost, ws.capture);
        if (e != hipSuccess) crc = hip_fail(e, "hipMemcpyAsync(flags)");
      }
      ws.stream = user;
      hipError_t e = hipStreamEndCapture(ws.capture, &g);
      if (crc) {
        if (g) (void)hipGraphDestroy(g);
        return crc;
      }
      if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
      GraphEntry ge;
      e = hipGraphInstantiate(&ge.exec, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
      ge.stages = batch;
      ge.generation = ws.generation;
      ge.epoch_span = ws.epoch_span;
      it = g_graphs.emplace(gk, ge).first;
    }
    it->second.last_use = ++g_graph_clock;
    ws.epoch_span = it->second.epoch_span;  // the passes after the graph continue its tags
    {
      OrderedLaunches order(dev, stream);
      if (order.status()) return order.status();
      KSORT_HIP(hipGraphLaunch(it->second.exec, stream));
    }
    KSORT_HIP(hipStreamSynchronize(stream));
    stage = it->second.stages;
    graphed = true;
  } else {
    if (d_offsets) {
      int64_t longest = n;
      if ((rc = longest_array(d_offsets, nseg, n, stream, &longest))) return rc;
      batch = predict_stages(longest, v->cutoff, v->tile());
    }
    rc = enqueue_prologue(ws, *v, dtype, d_data, n, d_offsets, nseg, d_pivots);
    if (rc) return rc;
  }

  size_t nev = 0;  // events of the pool used by this call
  std::vector<int> ev_stage;
  for (;;) {
    if (graphed) {
      graphed = false;  // flags were read back by the graph
    } else {
     {
      RoctxRange range(stage, batch, n);
      OrderedLaunches order(dev, stream);
      if (order.status()) return order.status();
      for (int b = 0; b < batch; ++b, ++stage) {
        if (epoch_wraps_before(stage, ws.epoch_span)) {
          rc = launch_clear_status(ws);
          if (rc) return rc;
        }
        if (prof) {
          while (ws.events.size() < nev + 2) {
            hipEvent_t e;
            KSORT_HIP(hipEventCreate(&e));
            ws.events.push_back(e);
          }
          KSORT_HIP(hipEventRecord(ws.events[nev], stream));
          rc = launch_stage(ws, *v, stage_args(ws, *v, stage, d_pivots, 1, 1), grid);
          KSORT_HIP(hipEventRecord(ws.events[nev + 1], stream));
          nev += 2;
          ev_stage.push_back(stage);
        } else {
          rc = launch_stage(ws, *v, stage_args(ws, *v, stage, d_pivots, 1, 1), grid);
        }
        if (rc) return rc;
      }
      KSORT_HIP(hipMemcpyAsync(ws.h_flags, ws.flags, sizeof(Flags), hipMemcpyDeviceToHost, stream));
     }
      KSORT_HIP(hipStreamSynchronize(stream));
    }
    const Flags f = *ws.h_flags;
    if ((rc = flags_error(f))) return rc;
    if (f.last_active < stage) {
      if (f.err) return fail(KSORT_EINVAL, "an array offset is outside [0, n_total] or decreasing");
      break;
    }
    // every level pass finishes at least one key per live segment
    if (stage > n + 64) return fail(KSORT_EINTERNAL, "level loop did not terminate");
    batch = more;
    more = std::min(64, 2 * more);
  }

  if (prof) {
    std::vector<int64_t> sk((size_t)ws.cap_stats * 2);
    KSORT_HIP(hipMemcpy(sk.data(), ws.stage_keys, sk.size() * sizeof(int64_t), hipMemcpyDeviceToHost));
    for (size_t k = 0; k < ev_stage.size(); ++k) {
      float ms = 0.f;
      KSORT_HIP(hipEventElapsedTime(&ms, ws.events[2 * k], ws.events[2 * k + 1]));
      ksort_level_record r;
      memset(&r, 0, sizeof r);
      r.call = call;
      r.dtype = dtype;
      r.stage = ev_stage[k];
      r.live_keys = ev_stage[k] < ws.cap_stats ? sk[2 * ev_stage[k]] : -1;
      r.finish_keys = ev_stage[k] < ws.cap_stats ? sk[2 * ev_stage[k] + 1] : -1;
      r.ms = ms;
      r.block = v->block;
      r.items = v->items;
      r.cutoff = v->cutoff;
      r.grid = grid;
      profile_push(r);
    }
  }
  return KSORT_OK;
}

// ---------------------------------------------------------------- static scratch
//
// Scratch for callers that cannot allocate: one file-scope device array per
// GPU, holding the descriptor lists, counters, flags, look-back words and
// the ping-pong keys of one sort.  Host code never uses the array's name as
// an address: the device address comes from hipGetSymbolAddress, once per
// device, with that device current.

constexpr size_t kStaticScratchBytes = KSORT_STATIC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char g_static_scratch[kStaticScratchBytes];

struct StaticSlot {
  std::mutex mu;
  bool ready = false;
  void* ptr = nullptr;  // this device's copy of g_static_scratch
  Workspace ws;
  Flags h_flags;        // flags are read back into this (pageable) word
};
constexpr int kMaxStaticDevices = 64;
static StaticSlot g_static[kMaxStaticDevices];

// Bytes of static scratch a sort of n keys with variant v takes.
static size_t static_bytes_for(const Variant& v, const Caps& c, int64_t n) {
  return align256(arena_bytes_for(c, (int)c.stats)) + align256((size_t)std::max<int64_t>(n, 1) * v.key_bytes);
}

// The largest n whose sort fits the static scratch (the variant chosen for
// each n as a plain sort would choose it).
static int64_t static_max_keys(int dtype) {
  int64_t lo = 1, hi = (int64_t)(kStaticScratchBytes / (dtype == KSORT_F64 ? 8 : 4)) + 1;
  while (hi - lo > 1) {
    const int64_t mid = lo + (hi - lo) / 2;
    const Variant* v = find_variant(dtype, nullptr, mid);
    if (static_bytes_for(*v, caps_for(*v, mid, 1, false), mid) <= kStaticScratchBytes)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

static int sort_static(int dtype, void* d_data, int64_t n, int64_t* d_pivot, hipStream_t stream) {
  if (dtype != KSORT_F64 && dtype != KSORT_F32) return fail(KSORT_EINVAL, "bad dtype");
  if (n < 0) return fail(KSORT_EINVAL, "negative size");
  if (n > 0 && !d_data) return fail(KSORT_EINVAL, "null data pointer");
  if (n <= 1) {
    if (d_pivot) {
      const int64_t fp = n == 0 ? -1 : 0;
      KSORT_HIP(hipMemcpyAsync(d_pivot, &fp, sizeof fp, hipMemcpyHostToDevice, stream));
      KSORT_HIP(hipStreamSynchronize(stream));
    }
    return KSORT_OK;
  }
  const Variant* v = find_variant(dtype, nullptr, n);
  const Caps c = caps_for(*v, n, 1, false);
  if (static_bytes_for(*v, c, n) > kStaticScratchBytes)
    return fail(KSORT_ETOOLARGE, "a sort of " + std::to_string(n) + " keys needs " +
                                     std::to_string(static_bytes_for(*v, c, n)) + " bytes of scratch; the static " +
                                     "scratch holds " + std::to_string(kStaticScratchBytes) + " (at most " +
                                     std::to_string(static_max_keys(dtype)) + " keys of this type)");
  int dev = 0;
  KSORT_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxStaticDevices) return fail(KSORT_EUNSUPPORTED, "device ordinal beyond the static slots");
  const DeviceInfo* di = nullptr;
  int rc = device_info(dev, &di);
  if (rc) return rc;
  if (!di->gfx950) return fail(KSORT_EUNSUPPORTED, "device " + std::to_string(dev) + " is " + di->arch + ", not gfx950");
  StaticSlot& sl = g_static[dev];
  std::lock_guard<std::mutex> lk(sl.mu);
  if (!sl.ready) {
    // set-up, once per device with that device current
    void* p = nullptr;
    KSORT_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(g_static_scratch)));
    sl.ptr = p;
    sl.ws.device = dev;
    sl.ws.user = sl.ptr;
    sl.ws.user_bytes = kStaticScratchBytes;
    sl.ws.h_flags = &sl.h_flags;
    sl.ws.own_h_flags = false;
    sl.ready = true;
  }
  // The lists keep the largest capacities of earlier calls; when those and
  // this call's keys do not fit together, lay the lists out for this call.
  Caps grown = sl.ws.caps;
  grown.live = std::max(grown.live, c.live);
  grown.tiles = std::max(grown.tiles, c.tiles);
  grown.fin = std::max(grown.fin, c.fin);
  grown.bufs = std::max(grown.bufs, c.bufs);
  grown.stats = std::max(grown.stats, c.stats);
  if (static_bytes_for(*v, grown, n) > kStaticScratchBytes) sl.ws.caps = Caps{};
  return sort_in(sl.ws, *v, *di, dtype, d_data, n, nullptr, 1, d_pivot, stream, false, false);
}

static int run_level(int dtype, const void* d_in, void* d_out, int64_t n, const int64_t* d_left,
                     const int64_t* d_len, int64_t nseg, int64_t* d_pivot, hipStream_t stream) {
  if (dtype != KSORT_F64 && dtype != KSORT_F32) return fail(KSORT_EINVAL, "bad dtype");
  if (n < 0 || nseg < 0) return fail(KSORT_EINVAL, "negative size");
  if (nseg == 0) return KSORT_OK;
  if (!d_in || !d_out || !d_left || !d_len || !d_pivot) return fail(KSORT_EINVAL, "null pointer");
  if (d_in == d_out) return fail(KSORT_EINVAL, "d_in and d_out must not overlap");
  if (nseg > 0x7ffffff0) return fail(KSORT_EINVAL, "too many segments");
  const Variant* v = find_variant(dtype, nullptr);
  int dev = 0;
  KSORT_HIP(hipGetDevice(&dev));
  const DeviceInfo* di = nullptr;
  int rc = device_info(dev, &di);
  if (rc) return rc;
  if (!di->gfx950) return fail(KSORT_EUNSUPPORTED, "device is " + di->arch + ", not gfx950");
  Workspace& ws = *workspace_for(dev, stream);
  std::lock_guard<std::mutex> lk(ws.mu);
  const Caps caps = caps_for(*v, n, nseg, true);
  rc = ws.reserve(caps, 0);
  ws.stats = false;
  if (rc) return rc;
  rc = launch_reset(ws);
  if (rc) return rc;
  InitArgs ia;
  memset(&ia, 0, sizeof ia);
  ia.sa = stage_args(ws, *v, 0, d_pivot, 0, 0);
  ia.pair.data = d_out;
  ia.pair.scratch = const_cast<void*>(d_in);
  ia.buf = 0;
  ia.root_base = 0;
  ia.n = n;
  ia.offsets = nullptr;
  ia.seg_left = d_left;
  ia.seg_len = d_len;
  ia.nseg = nseg;
  ia.level_mode = 1;
  ia.tile = v->tile();
  rc = launch_init(ws, *v, ia, nseg);
  if (rc) return rc;
  const int grid = stage_grid(*v, *di, ws.caps);
  {
    OrderedLaunches order(dev, stream);
    if (order.status()) return order.status();
    rc = launch_stage(ws, *v, stage_args(ws, *v, 0, d_pivot, 0, 0), grid);
  }
  if (rc) return rc;
  KSORT_HIP(hipMemcpyAsync(ws.h_flags, ws.flags, sizeof(Flags), hipMemcpyDeviceToHost, stream));
  KSORT_HIP(hipStreamSynchronize(stream));
  if ((rc = flags_error(*ws.h_flags))) return rc;
  if (ws.h_flags->err) return fail(KSORT_EINVAL, "a segment is outside [0, n) or has len < 1");
  return KSORT_OK;
}

}  // namespace ksort

// ============================================================== C ABI

using namespace ksort;

extern "C" {

int ksort_sort_ex(int dtype, void* d_data, int64_t n, int64_t* d_first_pivot, const ksort_tuning* tune,
                  void* stream) {
  return run_sort(dtype, d_data, n, nullptr, 1, d_first_pivot, tune, (hipStream_t)stream, false);
}

int ksort_sort_static(int dtype, void* d_data, int64_t n, int64_t* d_first_pivot, void* stream) {
  return sort_static(dtype, d_data, n, d_first_pivot, (hipStream_t)stream);
}

int ksort_f64(double* d_data, int64_t n, void* stream) {
  return run_sort(KSORT_F64, d_data, n, nullptr, 1, nullptr, nullptr, (hipStream_t)stream, false);
}

int ksort_f32(float* d_data, int64_t n, void* stream) {
  return run_sort(KSORT_F32, d_data, n, nullptr, 1, nullptr, nullptr, (hipStream_t)stream, false);
}

int ksort_partition_level(int dtype, const void* d_in, void* d_out, int64_t n, const int64_t* d_seg_left,
                          const int64_t* d_seg_len, int64_t nseg, int64_t* d_pivot, void* stream) {
  return run_level(dtype, d_in, d_out, n, d_seg_left, d_seg_len, nseg, d_pivot, (hipStream_t)stream);
}

int ksort_segmented(int dtype, void* d_packed, int64_t n_total, const int64_t* d_offsets, int64_t nseg,
                    int64_t* d_first_pivots, const ksort_tuning* tune, void* stream) {
  if (nseg < 0) return fail(KSORT_EINVAL, "negative nseg");
  if (nseg > 0 && !d_offsets) return fail(KSORT_EINVAL, "null offsets");
  if (n_total > 0 && !d_packed) return fail(KSORT_EINVAL, "null data pointer");
  return run_sort(dtype, d_packed, n_total, d_offsets, nseg, d_first_pivots, tune, (hipStream_t)stream, true);
}

int ksort_variants(int dtype, ksort_tuning* out, int cap) {
  if (dtype != KSORT_F64 && dtype != KSORT_F32) return fail(KSORT_EINVAL, "bad dtype");
  int cnt = 0;
  for (const auto& v : variants()) {
    if (v.dtype != dtype) continue;
    if (out && cnt < cap) {
      out[cnt].block = v.block;
      out[cnt].items = v.items;
      out[cnt].cutoff = v.cutoff;
      out[cnt].reserved = 0;
    }
    ++cnt;
  }
  return cnt;
}

int ksort_get_default(int dtype, ksort_tuning* out) {
  const Variant* v = find_variant(dtype, nullptr);
  if (!v || !out) return fail(KSORT_EINVAL, "bad dtype or null output");
  out->block = v->block;
  out->items = v->items;
  out->cutoff = v->cutoff;
  out->reserved = 0;
  return KSORT_OK;
}

int ksort_set_default(int dtype, const ksort_tuning* tune) { return set_default_variant(dtype, tune); }

int ksort_profile_enable(int on) {
  g_profile.store(on ? 1 : 0);
  return KSORT_OK;
}

int64_t ksort_profile_count(void) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  return (int64_t)g_prof.size();
}

int64_t ksort_profile_read(ksort_level_record* out, int64_t cap) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  const int64_t n = std::min<int64_t>(cap, (int64_t)g_prof.size());
  if (out && n > 0) memcpy(out, g_prof.data(), (size_t)n * sizeof(ksort_level_record));
  g_prof.clear();
  return n;
}

static size_t workspace_bytes_for(const Variant* v, int64_t n, int64_t nseg);

size_t ksort_workspace_bytes(int dtype, int64_t n, int64_t nseg) {
  if (n < 0 || nseg < 0) return 0;
  // the variant a single sort or a batch of this size would take
  const Variant* vs = find_variant(dtype, nullptr, n, kTuneSingle);
  const Variant* vb = find_variant(dtype, nullptr, n, kTuneBatch);
  if (!vs || !vb) return 0;
  return std::max(workspace_bytes_for(vs, n, nseg), workspace_bytes_for(vb, n, nseg));
}

static size_t workspace_bytes_for(const Variant* v, int64_t n, int64_t nseg) {
  // the larger of the sort's and the one-level pass's lists
  Caps c = caps_for(*v, n, nseg, false);
  const Caps cl = caps_for(*v, n, nseg, true);
  c.live = std::max(c.live, cl.live);
  c.tiles = std::max(c.tiles, cl.tiles);
  c.fin = std::max(c.fin, cl.fin);
  c.bufs = std::max(c.bufs, cl.bufs);
  c.stats = std::max(c.stats, cl.stats);
  return align256(arena_bytes_for(c, (int)c.stats)) + align256((size_t)std::max<int64_t>(n, 1) * v->key_bytes);
}

int ksort_set_workspace(void* d_ws, size_t bytes, void* stream) {
  if (d_ws && ((uintptr_t)d_ws % 256 != 0 || bytes < 4096))
    return fail(KSORT_EINVAL, "the workspace must be 256-byte aligned and at least 4096 bytes");
  int dev = 0;
  KSORT_HIP(hipGetDevice(&dev));
  Workspace& ws = *workspace_for(dev, (hipStream_t)stream);
  std::lock_guard<std::mutex> lk(ws.mu);
  {
    // captured graphs hold pointers into the old memory
    std::lock_guard<std::mutex> gl(g_graph_mu);
    for (auto it = g_graphs.begin(); it != g_graphs.end();) {
      if (it->first.first == &ws) {
        (void)hipGraphExecDestroy(it->second.exec);
        it = g_graphs.erase(it);
      } else {
        ++it;
      }
    }
  }
  return ws.use_memory(d_ws, bytes);
}

int ksort_release_workspaces(void) {
  {
    std::lock_guard<std::mutex> gl(g_graph_mu);
    for (auto& kv : g_graphs) (void)hipGraphExecDestroy(kv.second.exec);
    g_graphs.clear();
  }
  release_workspaces();
  release_exact_arenas();
  return KSORT_OK;
}

const char* ksort_strerror(int code) {
  switch (code) {
    case KSORT_OK: return "ok";
    case KSORT_EINVAL: return "invalid argument";
    case KSORT_ENOMEM: return "out of memory";
    case KSORT_EHIP: return "HIP runtime error";
    case KSORT_EUNSUPPORTED: return "unsupported device (gfx950 required)";
    case KSORT_ETOOLARGE: return "request exceeds the server budget";
    case KSORT_EAGAIN: return "server queue full";
    case KSORT_ECANCELLED: return "cancelled";
    case KSORT_ETIMEOUT: return "timed out";
    case KSORT_ENOTFOUND: return "unknown ticket";
    case KSORT_EINTERNAL: return "internal error";
    default: return "unknown error";
  }
}

const char* ksort_last_error(void) { return t_last_error.c_str(); }

const char* ksort_version(void) { return "ksort-mi355x 0.1 (gfx950)"; }

}  // extern "C"
