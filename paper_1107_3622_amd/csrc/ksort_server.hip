// Sort server with continuous batching.
//
// One scheduler thread per server.  Requests wait in a FIFO queue until their
// footprint fits the memory budget and an in-flight slot is free; an admitted
// request gets a slot (its buffer pair: the caller's array and a piece of the
// server's scratch arena) and its whole array joins the lists of the current
// stage of its key type's lane.  Every scheduler tick launches one stage per
// lane with work: one level pass (partition + LDS finish) over the segments of
// all admitted requests together, exactly the kernels of the plain sort.  The
// device keeps a count of outstanding segments per slot and records the stage
// at which it drops to zero; after each tick the host reads those stages back
// and completes the finished requests.  New requests are admitted at every
// tick, so they overlap with requests already in flight.
#include <hip/hip_runtime.h>

#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "ksort.h"
#include "ksort_engine.h"
#include "ksort_epoch.h"
#include "ksort_sched.h"

namespace ksort {

static double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

struct Lane {
  int dtype = 0;
  const Variant* v = nullptr;
  hipStream_t stream = nullptr;
  Workspace ws;
  int64_t stage = 0;              // passes launched on this lane (64-bit: a busy lane never wraps it)
  int grid = 1;
  int active = 0;                 // admitted, unfinished requests
  std::vector<uint64_t> slot_req; // slot -> request id (0 = free)
  int64_t* d_pivot = nullptr;     // per slot
  int32_t* h_done = nullptr;      // pinned copies
  int64_t* h_pivot = nullptr;
  Flags* h_flags = nullptr;
};

}  // namespace ksort

struct ksort_server {
  int device = 0;
  int max_inflight = 0;
  size_t budget = 0;
  ksort::Scheduler sched;
  ksort::RangeAlloc scratch_alloc;
  void* scratch = nullptr;
  ksort::Lane lanes[2];
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::thread th;
  bool stop = false;
  int thread_error = 0;
  std::string thread_error_msg;
  std::string last_failure;  // detail of the latest failed request (device check)
  double busy_since = -1;
  ksort_server(size_t b, int mi) : max_inflight(mi), budget(b), sched(b, mi, 1u << 20), scratch_alloc(b / 2) {}
};

namespace ksort {

static size_t footprint_of(const Variant& v, int64_t n) {
  const size_t kb = v.key_bytes;
  // data + ping-pong scratch + descriptors and look-back words of its tiles
  return 2 * (size_t)n * kb + 96 * ((size_t)n / (size_t)v.tile() + 4);
}

static int lane_init(ksort_server* s, Lane& L, int dtype) {
  L.dtype = dtype;
  L.v = find_variant(dtype, nullptr);
  const DeviceInfo* di = nullptr;
  int rc = device_info(s->device, &di);
  if (rc) return rc;
  if (!di->gfx950) return fail(KSORT_EUNSUPPORTED, "device is " + di->arch + ", not gfx950");
  KSORT_HIP(hipStreamCreateWithFlags(&L.stream, hipStreamNonBlocking));
  L.ws.device = s->device;
  L.ws.stream = L.stream;
  L.ws.cap_stats = 1;
  L.ws.epoch_span = epoch_span_setting();
  const int64_t n_eff = (int64_t)(s->budget / (2 * L.v->key_bytes));
  Caps c = caps_for(*L.v, n_eff, s->max_inflight, false);
  c.live += s->max_inflight;
  c.tiles += s->max_inflight;
  c.fin += s->max_inflight;
  c.bufs = s->max_inflight;
  rc = L.ws.reserve(c, 0);
  if (rc) return rc;
  L.grid = stage_grid(*L.v, *di, L.ws.caps);
  L.slot_req.assign((size_t)s->max_inflight, 0);
  KSORT_HIP(hipMalloc((void**)&L.d_pivot, (size_t)s->max_inflight * sizeof(int64_t)));
  KSORT_HIP(hipHostMalloc((void**)&L.h_done, (size_t)s->max_inflight * sizeof(int32_t), hipHostMallocDefault));
  KSORT_HIP(hipHostMalloc((void**)&L.h_pivot, (size_t)s->max_inflight * sizeof(int64_t), hipHostMallocDefault));
  KSORT_HIP(hipHostMalloc((void**)&L.h_flags, sizeof(Flags), hipHostMallocDefault));
  // clear counters and look-back words once; the stage counter then runs on
  KSORT_HIP(hipMemsetAsync(L.ws.done_stage, 0xff, (size_t)s->max_inflight * sizeof(int32_t), L.stream));
  rc = launch_reset(L.ws);
  if (rc) return rc;
  KSORT_HIP(hipStreamSynchronize(L.stream));
  return KSORT_OK;
}

static void lane_free(Lane& L) {
  if (L.stream) (void)hipStreamSynchronize(L.stream);
  if (L.d_pivot) (void)hipFree(L.d_pivot);
  if (L.h_done) (void)hipHostFree(L.h_done);
  if (L.h_pivot) (void)hipHostFree(L.h_pivot);
  if (L.h_flags) (void)hipHostFree(L.h_flags);
  if (L.stream) (void)hipStreamDestroy(L.stream);
  L.d_pivot = nullptr;
  L.h_done = nullptr;
  L.h_pivot = nullptr;
  L.h_flags = nullptr;
  L.stream = nullptr;
}

// Pass s of a lane runs as kernel pass kernel_stage(s) with the look-back
// tag of s itself (ksort_epoch.h).  A request's completion is seen after the
// tick in which it completes, so its level count follows from the host's s.
static StageArgs server_args(Lane& L) {
  StageArgs a = stage_args(L.ws, *L.v, kernel_stage(L.stage), L.d_pivot, 1, 1);
  a.epoch = epoch_of(L.stage, L.ws.epoch_span);
  a.pending = L.ws.pending;
  a.done_stage = L.ws.done_stage;
  a.stage_keys = nullptr;
  // Request producers run kernels while the server's passes run, so a
  // workgroup of a pass may wait for slots they hold: every work ticket comes
  // from the counter, so no tile waits for a workgroup that has not started.
  a.fixed_first = 0;
  // Every finish task runs in the pass that lists it: a busy server always
  // has partition tiles, and deferring finish work to a pass without tiles
  // would hold requests back for as long as new ones keep arriving.
  a.fin_run = 0x7fffffff;
  return a;
}

// Queue the admission of request r into lane L's current stage.
static int lane_admit(ksort_server* s, Lane& L, Request& r) {
  InitArgs ia;
  memset(&ia, 0, sizeof ia);
  ia.sa = server_args(L);
  ia.pair.data = r.data;
  ia.pair.scratch = (char*)s->scratch + r.scratch_off;
  ia.buf = r.slot;
  ia.root_base = r.slot;
  ia.n = r.n;
  ia.nseg = 1;
  ia.level_mode = 0;
  ia.tile = L.v->tile();
  L.slot_req[(size_t)r.slot] = r.id;
  r.admit_stage = L.stage;
  ++L.active;
  return launch_init(L.ws, *L.v, ia, 1);
}

// After a failed device check the lane's lists may be incomplete; every
// request on it has been failed.  Clearing its counters, flags, look-back
// words and per-slot states lets it serve new requests.
static int lane_recover(Lane& L) {
  const size_t slots = L.slot_req.size();
  KSORT_HIP(hipMemsetAsync(L.ws.done_stage, 0xff, slots * sizeof(int32_t), L.stream));
  KSORT_HIP(hipMemsetAsync(L.ws.pending, 0, slots * sizeof(int32_t), L.stream));
  int rc = launch_reset(L.ws);
  if (rc) return rc;
  KSORT_HIP(hipStreamSynchronize(L.stream));
  return KSORT_OK;
}

// One tick of a lane: one stage over every admitted request, then the read
// back of per-slot completion stages and pivots.
static int lane_launch(ksort_server* s, Lane& L) {
  if (epoch_wraps_before(L.stage, L.ws.epoch_span)) {
    // The look-back tags wrap: clear the words and nothing else.  The stage
    // counters, lists and per-slot counts hold the work of the requests in
    // flight and go on unchanged.
    int rc = launch_clear_status(L.ws);
    if (rc) return rc;
  }
  {
    OrderedLaunches order(s->device, L.stream);
    if (order.status()) return order.status();
    int rc = launch_stage(L.ws, *L.v, server_args(L), L.grid);
    if (rc) return rc;
  }
  const size_t slots = (size_t)s->max_inflight;
  KSORT_HIP(hipMemcpyAsync(L.h_done, L.ws.done_stage, slots * sizeof(int32_t), hipMemcpyDeviceToHost, L.stream));
  KSORT_HIP(hipMemcpyAsync(L.h_pivot, L.d_pivot, slots * sizeof(int64_t), hipMemcpyDeviceToHost, L.stream));
  KSORT_HIP(hipMemcpyAsync(L.h_flags, L.ws.flags, sizeof(Flags), hipMemcpyDeviceToHost, L.stream));
  ++L.stage;
  return KSORT_OK;
}

static void server_loop(ksort_server* s) {
  (void)hipSetDevice(s->device);
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    // admission
    const double t = now_s();
    std::vector<Request*> adm = s->sched.admit(t, [&](Request& r) {
      size_t off = 0;
      if (!s->scratch_alloc.alloc(r.scratch_bytes, &off)) return false;
      r.scratch_off = off;
      return true;
    });
    const bool busy = s->lanes[0].active + s->lanes[1].active + (int)adm.size() > 0;
    if (!busy) {
      if (s->busy_since >= 0) {
        s->sched.stats().busy_s += t - s->busy_since;
        s->busy_since = -1;
      }
      if (s->stop) break;
      s->cv_work.wait_for(lk, std::chrono::milliseconds(50));
      continue;
    }
    if (s->busy_since < 0) s->busy_since = t;
    int rc = KSORT_OK;
    for (Request* r : adm) {
      if (rc == KSORT_OK) rc = lane_admit(s, s->lanes[r->dtype], *r);
    }
    // launch one stage per lane with work
    bool launched[2] = {false, false};
    lk.unlock();
    for (int d = 0; d < 2 && rc == KSORT_OK; ++d) {
      Lane& L = s->lanes[d];
      if (L.active > 0) {
        rc = lane_launch(s, L);
        launched[d] = rc == KSORT_OK;
      }
    }
    for (int d = 0; d < 2; ++d) {
      if (launched[d]) {
        hipError_t e = hipStreamSynchronize(s->lanes[d].stream);
        if (e != hipSuccess && rc == KSORT_OK) rc = hip_fail(e, "hipStreamSynchronize(server)");
      }
    }
    lk.lock();
    s->sched.stats().ticks++;
    const double t2 = now_s();
    // completions
    for (int d = 0; d < 2; ++d) {
      Lane& L = s->lanes[d];
      if (!launched[d] && rc == KSORT_OK) continue;
      const bool lane_bad = rc != KSORT_OK || (launched[d] && L.h_flags->overflow);
      if (lane_bad) {
        if (rc == KSORT_OK) (void)flags_error(*L.h_flags);
        s->last_failure = ksort_last_error();
      }
      for (size_t k = 0; k < L.slot_req.size(); ++k) {
        const uint64_t id = L.slot_req[k];
        if (!id) continue;
        Request* r = s->sched.find(id);
        if (!r) continue;
        if (lane_bad) {
          s->scratch_alloc.release(r->scratch_off, r->scratch_bytes);
          s->sched.complete(id, rc != KSORT_OK ? rc : KSORT_EINTERNAL, t2, -1, (int)(L.stage - r->admit_stage));
          L.slot_req[k] = 0;
          --L.active;
        } else if (L.h_done[k] >= 0) {
          s->scratch_alloc.release(r->scratch_off, r->scratch_bytes);
          // completed in the pass just read back, pass L.stage - 1
          s->sched.complete(id, kReqDone, t2, L.h_pivot[k], (int)(L.stage - r->admit_stage));
          L.slot_req[k] = 0;
          --L.active;
        }
      }
      if (lane_bad && rc == KSORT_OK) {
        const int rr = lane_recover(L);
        if (rr != KSORT_OK) rc = rr;
      }
    }
    if (rc != KSORT_OK) {
      s->thread_error = rc;
      s->thread_error_msg = ksort_last_error();
    }
    s->cv_done.notify_all();
  }
  s->cv_done.notify_all();
}

}  // namespace ksort

using namespace ksort;

extern "C" {

ksort_server* ksort_server_create(size_t hbm_budget_bytes, int max_inflight, int device) {
  if (hbm_budget_bytes < (1u << 20) || max_inflight < 1 || max_inflight > (1 << 20) || device < 0) {
    fail(KSORT_EINVAL, "budget must be >= 1 MiB and 1 <= max_inflight <= 2^20");
    return nullptr;
  }
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device >= ndev) {
    fail(KSORT_EINVAL, "no such device");
    return nullptr;
  }
  int prev = 0;
  (void)hipGetDevice(&prev);
  if (hipSetDevice(device) != hipSuccess) {
    fail(KSORT_EHIP, "hipSetDevice failed");
    return nullptr;
  }
  auto s = std::make_unique<ksort_server>(hbm_budget_bytes, max_inflight);
  s->device = device;
  int rc = KSORT_OK;
  hipError_t e = hipMalloc(&s->scratch, std::max<size_t>(hbm_budget_bytes / 2, 256));
  if (e != hipSuccess) rc = hip_fail(e, "hipMalloc(server scratch)");
  for (int d = 0; d < 2 && rc == KSORT_OK; ++d) rc = lane_init(s.get(), s->lanes[d], d);
  (void)hipSetDevice(prev);
  if (rc != KSORT_OK) {
    for (int d = 0; d < 2; ++d) lane_free(s->lanes[d]);
    if (s->scratch) (void)hipFree(s->scratch);
    return nullptr;
  }
  ksort_server* raw = s.release();
  raw->th = std::thread(server_loop, raw);
  return raw;
}

int ksort_server_submit(ksort_server* s, int dtype, void* d_data, int64_t n, uint64_t* ticket) {
  if (!s || !ticket) return fail(KSORT_EINVAL, "null server or ticket");
  if (dtype != KSORT_F64 && dtype != KSORT_F32) return fail(KSORT_EINVAL, "bad dtype");
  if (n < 0 || (n > 0 && !d_data)) return fail(KSORT_EINVAL, "bad array");
  if (n > ((int64_t)1 << 31) - 1) return fail(KSORT_ETOOLARGE, "more than 2^31-1 keys");
  const Variant& v = *s->lanes[dtype].v;
  const size_t fp = footprint_of(v, n);
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->stop) return fail(KSORT_ECANCELLED, "server is shutting down");
  int rc = s->sched.submit(dtype, d_data, n, fp, (size_t)n * v.key_bytes, now_s(), ticket);
  if (rc == kSchedTooLarge) return fail(KSORT_ETOOLARGE, "request footprint exceeds the budget");
  if (rc == kSchedAgain) return fail(KSORT_EAGAIN, "queue full");
  if (rc) return fail(KSORT_EINVAL, "bad request");
  if (n == 0) {
    s->sched.complete_queued_trivially(*ticket, now_s());
    s->cv_done.notify_all();
  } else {
    s->cv_work.notify_one();
  }
  return KSORT_OK;
}

int ksort_server_poll(ksort_server* s, uint64_t ticket, int* state) {
  if (!s || !state) return fail(KSORT_EINVAL, "null argument");
  std::lock_guard<std::mutex> lk(s->mu);
  const Request* r = s->sched.find(ticket);
  if (!r) return fail(KSORT_ENOTFOUND, "unknown ticket");
  *state = r->state == kReqRunning ? 0 : r->state;
  return KSORT_OK;
}

int ksort_server_wait(ksort_server* s, uint64_t ticket, double timeout_s) {
  if (!s) return fail(KSORT_EINVAL, "null server");
  std::unique_lock<std::mutex> lk(s->mu);
  auto done = [&] {
    const Request* r = s->sched.find(ticket);
    return !r || (r->state != kReqQueued && r->state != kReqRunning);
  };
  if (timeout_s < 0) {
    s->cv_done.wait(lk, done);
  } else if (!s->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), done)) {
    return fail(KSORT_ETIMEOUT, "wait timed out");
  }
  const Request* r = s->sched.find(ticket);
  if (!r) return fail(KSORT_ENOTFOUND, "unknown ticket");
  if (r->state == kReqDone) return KSORT_OK;
  if (r->state == KSORT_ECANCELLED) return fail(r->state, "request cancelled");
  return fail(r->state, "request failed: " + (s->last_failure.empty() ? std::string("no detail") : s->last_failure));
}

int ksort_server_cancel(ksort_server* s, uint64_t ticket) {
  if (!s) return fail(KSORT_EINVAL, "null server");
  std::lock_guard<std::mutex> lk(s->mu);
  const int rc = s->sched.cancel(ticket, now_s());
  if (rc == kSchedNotFound) return fail(KSORT_ENOTFOUND, "unknown ticket");
  if (rc == kSchedAgain) return fail(KSORT_EAGAIN, "request already admitted; it will complete");
  s->cv_done.notify_all();
  return KSORT_OK;
}

int ksort_server_result(ksort_server* s, uint64_t ticket, ksort_request_info* out) {
  if (!s || !out) return fail(KSORT_EINVAL, "null argument");
  std::lock_guard<std::mutex> lk(s->mu);
  const Request* r = s->sched.find(ticket);
  if (!r) return fail(KSORT_ENOTFOUND, "unknown ticket");
  memset(out, 0, sizeof *out);
  out->n = r->n;
  out->dtype = r->dtype;
  out->state = r->state == kReqRunning ? 0 : r->state;
  out->first_pivot = r->state == kReqDone ? (r->n == 0 ? -1 : r->first_pivot) : -1;
  out->t_submit_s = r->t_submit;
  out->t_admit_s = r->t_admit;
  out->t_done_s = r->t_done;
  out->levels = r->levels;
  return KSORT_OK;
}

int ksort_server_stats(ksort_server* s, ksort_server_stats_t* out) {
  if (!s || !out) return fail(KSORT_EINVAL, "null argument");
  std::lock_guard<std::mutex> lk(s->mu);
  const SchedStats& st = s->sched.stats();
  memset(out, 0, sizeof *out);
  out->submitted = st.submitted;
  out->admitted = st.admitted;
  out->completed = st.completed;
  out->rejected = st.rejected;
  out->cancelled = st.cancelled;
  out->failed = st.failed;
  out->keys_completed = st.keys_completed;
  out->ticks = st.ticks;
  out->busy_s = st.busy_s + (s->busy_since >= 0 ? now_s() - s->busy_since : 0.0);
  out->p50_latency_s = Scheduler::percentile(st.latencies, 0.50);
  out->p99_latency_s = Scheduler::percentile(st.latencies, 0.99);
  double sum = 0;
  for (double x : st.latencies) sum += x;
  out->mean_latency_s = st.latencies.empty() ? 0.0 : sum / (double)st.latencies.size();
  out->inflight_now = s->sched.inflight();
  out->queued_now = (int64_t)s->sched.queued();
  out->budget_used_bytes = (int64_t)s->sched.used();
  return KSORT_OK;
}

void ksort_server_destroy(ksort_server* s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    s->sched.cancel_all_queued(now_s());
  }
  s->cv_work.notify_all();
  if (s->th.joinable()) s->th.join();
  int prev = 0;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(s->device);
  for (int d = 0; d < 2; ++d) lane_free(s->lanes[d]);
  if (s->scratch) (void)hipFree(s->scratch);
  (void)hipSetDevice(prev);
  delete s;
}

}  // extern "C"
