// Request bookkeeping of the sort server: FIFO admission under a memory
// budget and an in-flight cap, a first-fit sub-allocator for ping-pong
// scratch, request states and latency statistics.  Pure C++ (no HIP), so the
// policy can be tested on the host on its own.
#pragma once

#include <stdint.h>

#include <algorithm>
#include <cmath>
#include <deque>
#include <functional>
#include <iterator>
#include <map>
#include <vector>

namespace ksort {

// request states as reported by ksort_server_poll (negative = error)
constexpr int kReqQueued = 0;
constexpr int kReqDone = 1;
constexpr int kReqRunning = 2;

// error codes mirrored from ksort.h so this header stands alone
constexpr int kSchedOk = 0;
constexpr int kSchedInval = -1;
constexpr int kSchedTooLarge = -5;
constexpr int kSchedAgain = -6;
constexpr int kSchedCancelled = -7;
constexpr int kSchedNotFound = -9;

struct Request {
  uint64_t id = 0;
  int dtype = 0;
  void* data = nullptr;
  int64_t n = 0;
  size_t footprint = 0;      // bytes charged to the budget while admitted
  size_t scratch_bytes = 0;  // ping-pong scratch needed
  int state = kReqQueued;
  double t_submit = 0, t_admit = 0, t_done = 0;
  int64_t first_pivot = -1;
  int levels = 0;
  int slot = -1;             // buffer-pair slot while admitted
  size_t scratch_off = 0;    // offset of its scratch in the arena
  int64_t admit_stage = 0;  // server pass at which it joined its lane
};

// First-fit allocator of [0, size) with coalescing of free ranges.
class RangeAlloc {
 public:
  explicit RangeAlloc(size_t size = 0, size_t align = 256) : size_(size), align_(align) {
    if (size) free_[0] = size;
  }
  bool alloc(size_t bytes, size_t* off) {
    bytes = round(bytes ? bytes : 1);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        *off = it->first;
        const size_t rest = it->second - bytes;
        const size_t start = it->first + bytes;
        free_.erase(it);
        if (rest) free_[start] = rest;
        used_ += bytes;
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = round(bytes ? bytes : 1);
    used_ -= bytes;
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t used() const { return used_; }
  size_t size() const { return size_; }
  size_t free_ranges() const { return free_.size(); }

 private:
  size_t round(size_t b) const { return (b + align_ - 1) / align_ * align_; }
  size_t size_, align_, used_ = 0;
  std::map<size_t, size_t> free_;
};

struct SchedStats {
  int64_t submitted = 0, admitted = 0, completed = 0, rejected = 0, cancelled = 0, failed = 0;
  int64_t keys_completed = 0;
  int64_t ticks = 0;
  double busy_s = 0;
  std::vector<double> latencies;
};

// FIFO admission: a queued request is admitted when its footprint fits the
// remaining budget, an in-flight slot is free and `reserve` (the scratch
// allocation) succeeds; admission stops at the first request that does not
// fit, so requests are admitted in submission order.
class Scheduler {
 public:
  Scheduler(size_t budget, int max_inflight, size_t max_queue)
      : budget_(budget), max_queue_(max_queue) {
    for (int s = max_inflight - 1; s >= 0; --s) free_slots_.push_back(s);
  }

  int submit(int dtype, void* data, int64_t n, size_t footprint, size_t scratch_bytes, double now, uint64_t* id) {
    if (n < 0 || (dtype != 0 && dtype != 1)) return kSchedInval;
    if (footprint > budget_) {
      ++st_.rejected;
      return kSchedTooLarge;
    }
    if (queue_.size() >= max_queue_) {
      ++st_.rejected;
      return kSchedAgain;
    }
    Request r;
    r.id = next_id_++;
    r.dtype = dtype;
    r.data = data;
    r.n = n;
    r.footprint = footprint;
    r.scratch_bytes = scratch_bytes;
    r.t_submit = now;
    reqs_[r.id] = r;
    queue_.push_back(r.id);
    ++st_.submitted;
    *id = r.id;
    return kSchedOk;
  }

  // Admits in FIFO order; returns the admitted requests (state -> running).
  std::vector<Request*> admit(double now, const std::function<bool(Request&)>& reserve) {
    std::vector<Request*> out;
    while (!queue_.empty()) {
      Request& r = reqs_[queue_.front()];
      if (free_slots_.empty() || used_ + r.footprint > budget_) break;
      if (!reserve(r)) break;
      queue_.pop_front();
      r.slot = free_slots_.back();
      free_slots_.pop_back();
      r.state = kReqRunning;
      r.t_admit = now;
      used_ += r.footprint;
      ++inflight_;
      ++st_.admitted;
      out.push_back(&r);
    }
    return out;
  }

  // A running request finished with `status` (kReqDone or a negative code).
  void complete(uint64_t id, int status, double now, int64_t pivot, int levels) {
    auto it = reqs_.find(id);
    if (it == reqs_.end() || it->second.state != kReqRunning) return;
    Request& r = it->second;
    r.state = status;
    r.t_done = now;
    r.first_pivot = pivot;
    r.levels = levels;
    used_ -= r.footprint;
    free_slots_.push_back(r.slot);
    --inflight_;
    if (status == kReqDone) {
      ++st_.completed;
      st_.keys_completed += r.n;
      st_.latencies.push_back(r.t_done - r.t_submit);
    } else {
      ++st_.failed;
    }
  }

  // Completes a request that needs no device work (n == 0).
  void complete_queued_trivially(uint64_t id, double now) {
    auto it = reqs_.find(id);
    if (it == reqs_.end() || it->second.state != kReqQueued) return;
    queue_.erase(std::find(queue_.begin(), queue_.end(), id));
    it->second.state = kReqDone;
    it->second.t_admit = it->second.t_done = now;
    ++st_.completed;
    st_.latencies.push_back(0.0);
  }

  int cancel(uint64_t id, double now) {
    auto it = reqs_.find(id);
    if (it == reqs_.end()) return kSchedNotFound;
    Request& r = it->second;
    if (r.state != kReqQueued) return r.state == kReqRunning ? kSchedAgain : kSchedOk;
    queue_.erase(std::find(queue_.begin(), queue_.end(), id));
    r.state = kSchedCancelled;
    r.t_done = now;
    ++st_.cancelled;
    return kSchedOk;
  }

  void cancel_all_queued(double now) {
    while (!queue_.empty()) cancel(queue_.front(), now);
  }

  const Request* find(uint64_t id) const {
    auto it = reqs_.find(id);
    return it == reqs_.end() ? nullptr : &it->second;
  }
  Request* find(uint64_t id) {
    auto it = reqs_.find(id);
    return it == reqs_.end() ? nullptr : &it->second;
  }

  static double percentile(std::vector<double> v, double q) {
    if (v.empty()) return 0.0;
    std::sort(v.begin(), v.end());
    const double pos = q * (double)(v.size() - 1);
    const size_t lo = (size_t)std::floor(pos), hi = (size_t)std::ceil(pos);
    return v[lo] + (v[hi] - v[lo]) * (pos - (double)lo);
  }

  size_t used() const { return used_; }
  size_t budget() const { return budget_; }
  int inflight() const { return inflight_; }
  size_t queued() const { return queue_.size(); }
  SchedStats& stats() { return st_; }
  const SchedStats& stats() const { return st_; }

 private:
  size_t budget_;
  size_t max_queue_;
  size_t used_ = 0;
  int inflight_ = 0;
  uint64_t next_id_ = 1;
  std::map<uint64_t, Request> reqs_;
  std::deque<uint64_t> queue_;
  std::vector<int> free_slots_;
  SchedStats st_;
};

}  // namespace ksort
