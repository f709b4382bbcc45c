// Host-side level driver of the K-sort library (internal C++ interface,
// shared by the C ABI in ksort_lib.hip and the server in ksort_server.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>
#include <string>
#include <vector>

#include "ksort.h"
#include "ksort_types.h"

namespace ksort {

// thread-local error detail
void set_error(const std::string& msg);
int fail(int code, const std::string& msg);
int hip_fail(hipError_t e, const char* what);

#define KSORT_HIP(call)                                  \
  do {                                                   \
    hipError_t e_ = (call);                              \
    if (e_ != hipSuccess) return hip_fail(e_, #call);    \
  } while (0)

// A compiled kernel variant.
struct Variant {
  int dtype;
  int block, items, cutoff;
  const void* stage;      // stage_kernel<T, BLOCK, ITEMS, CUT>
  hipError_t (*launch)(const StageArgs& a, int grid, hipStream_t stream);  // enqueues it
  size_t key_bytes;
  int tile() const { return block * items; }
};

const std::vector<Variant>& variants();
// What a tuned choice applies to: single arrays of about n keys, or packed
// batches of about n keys in all.
enum TuneKind { kTuneSingle = 0, kTuneBatch = 1 };
// Explicit `tune` if given; otherwise the autotuned variant for inputs of
// about n keys of that kind, else the default for the key type.
const Variant* find_variant(int dtype, const ksort_tuning* tune, int64_t n = -1, int kind = kTuneSingle,
                            bool use_tuned = true);
bool tuned_for(int dtype, int64_t n, int kind, ksort_tuning* out);
int set_default_variant(int dtype, const ksort_tuning* tune);

struct DeviceInfo {
  int ordinal = -1;
  int cus = 0;
  bool gfx950 = false;
  std::string arch;
  std::vector<int> occupancy;  // blocks per CU, indexed like variants()
};
int device_info(int ordinal, const DeviceInfo** out);

// Capacities of the descriptor lists for one run.
struct Caps {
  int64_t live = 0, tiles = 0, fin = 0, bufs = 1;
  int64_t stats = 256;  // level passes whose key counts are kept for profiling
};
Caps caps_for(const Variant& v, int64_t n, int64_t nseg, bool level_mode);

// Device workspace: descriptor lists, counters, flags, look-back words and
// the ping-pong scratch.  One per (device, stream) for the C ABI calls; the
// server owns its own.
struct Workspace {
  int device = -1;
  hipStream_t stream = nullptr;
  void* arena = nullptr;
  size_t arena_bytes = 0;
  void* scratch = nullptr;
  size_t scratch_bytes = 0;
  Caps caps;
  int cap_stats = 256;
  StageCtr* ctr = nullptr;
  Flags* flags = nullptr;
  Seg* live[2] = {nullptr, nullptr};
  int32_t* tilemap[2] = {nullptr, nullptr};
  Seg* fin[2] = {nullptr, nullptr};
  uint64_t* status = nullptr;
  int64_t* stage_keys = nullptr;
  bool stats = false;          // this run keeps per-level key counts (profiling)
  int32_t* pending = nullptr;
  int32_t* done_stage = nullptr;
  uint32_t epoch = 0;         // last epoch used
  int64_t epoch_span = (1 << 22) - 1;  // look-back tags of this run (see ksort_epoch.h)
  uint64_t generation = 0;    // bumped whenever the arena or the scratch is laid out anew
  Flags* h_flags = nullptr;   // pinned readback (or memory the owner of the workspace provides)
  bool own_h_flags = true;    // h_flags was allocated by reserve() and is freed with the workspace
  hipStream_t capture = nullptr;  // private stream used only to record graphs
  std::vector<hipEvent_t> events; // pool for per-level timing (profiling mode)
  void* user = nullptr;        // caller's device memory (ksort_set_workspace), or null
  size_t user_bytes = 0;
  std::mutex mu;
  ~Workspace();
  // make room for a run; scratch_keys * key_bytes bytes of scratch
  int reserve(const Caps& c, size_t scratch_bytes_needed);
  // frees the library's own memory and hands the workspace d (or, for null,
  // memory the library allocates again); the caller holds mu
  int use_memory(void* d, size_t bytes);
  uint32_t next_epoch();      // clears the look-back words when the tag wraps
};

Workspace* workspace_for(int device, hipStream_t stream);
void release_workspaces();
void release_exact_arenas();  // scratch of the literal-arrangement calls

// Arguments of one stage launch built from a workspace.
StageArgs stage_args(Workspace& ws, const Variant& v, int stage, int64_t* pivot_out, int pivot_relative,
                     int emit_children);

// Error for a flag word read back after a batch of passes (KSORT_OK if the
// device checks passed); a timed-out look-back wait names its pass, tile and
// predecessor.
int flags_error(const Flags& f);

// Launch helpers (asynchronous on ws.stream).
// Stage kernels of this library never run concurrently on one device (their
// first work items are fixed per workgroup; see the stage kernel): each
// batch of stage launches waits for the previous batch on the device,
// whatever stream it was enqueued on.  Hold an OrderedLaunches while
// enqueuing a batch; its destructor marks the batch's end.
class OrderedLaunches {
 public:
  OrderedLaunches(int device, hipStream_t stream);
  ~OrderedLaunches();
  OrderedLaunches(const OrderedLaunches&) = delete;
  OrderedLaunches& operator=(const OrderedLaunches&) = delete;
  int status() const { return rc_; }
  struct Order;

 private:
  Order* o_;
  hipStream_t stream_;
  int rc_ = 0;
};

int launch_reset(Workspace& ws);
int launch_clear_status(Workspace& ws);  // the look-back words only
int launch_init(Workspace& ws, const Variant& v, const InitArgs& ia, int64_t nblocks);
int launch_stage(Workspace& ws, const Variant& v, const StageArgs& a, int grid);
int stage_grid(const Variant& v, const DeviceInfo& di, const Caps& c);

// Polls a look-back wait makes before it gives up (KSORT_SPIN_LIMIT, or 2^22).
uint32_t spin_limit_setting();

// Predicted number of level passes for n keys (used to size launch batches).
int predict_stages(int64_t n, int cutoff, int tile);

// Whole sort of one packed buffer (single array when offsets == nullptr).
int run_sort(int dtype, void* d_data, int64_t n, const int64_t* d_offsets, int64_t nseg,
             int64_t* d_pivots, const ksort_tuning* tune, hipStream_t stream, bool use_graph);

// Profiling records
bool profiling_on();
void profile_push(const ksort_level_record& r);
int64_t next_call_id();

}  // namespace ksort
