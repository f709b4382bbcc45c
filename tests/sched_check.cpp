// Host-only checks of the sort server's admission policy and scratch
// allocator (no GPU): FIFO admission under a memory budget and an in-flight
// cap, rejection of requests that can never fit, cancellation of queued
// requests, latency percentiles, first-fit allocation with coalescing.
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "ksort_sched.h"

using namespace ksort;

static int failures = 0;
#define CHECK(c)                                                   \
  do {                                                             \
    if (!(c)) {                                                    \
      std::fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #c); \
      ++failures;                                                  \
    }                                                              \
  } while (0)

static void range_alloc() {
  RangeAlloc ra(4096, 256);
  size_t a = 0, b = 0, c = 0, d = 0;
  CHECK(ra.alloc(100, &a) && a == 0);    // rounded up to 256
  CHECK(ra.alloc(256, &b) && b == 256);
  CHECK(ra.alloc(1000, &c) && c == 512);  // 1024 bytes
  CHECK(ra.used() == 256 + 256 + 1024);
  CHECK(!ra.alloc(4096, &d));
  ra.release(b, 256);                     // hole at [256, 512)
  CHECK(ra.alloc(200, &d) && d == 256);   // first fit reuses the hole
  ra.release(d, 200);
  ra.release(a, 100);                     // [0, 512) coalesces
  ra.release(c, 1000);                    // everything free again: one range
  CHECK(ra.used() == 0 && ra.free_ranges() == 1);
  CHECK(ra.alloc(4096, &d) && d == 0);
}

static void scheduler() {
  Scheduler s(1000, 2, 5);
  uint64_t id[8] = {};
  CHECK(s.submit(0, nullptr, 10, 400, 0, 0.0, &id[0]) == kSchedOk);
  CHECK(s.submit(1, nullptr, 10, 400, 0, 0.1, &id[1]) == kSchedOk);
  CHECK(s.submit(0, nullptr, 10, 700, 0, 0.2, &id[2]) == kSchedOk);
  CHECK(s.submit(0, nullptr, 10, 1001, 0, 0.3, &id[3]) == kSchedTooLarge);  // never fits
  CHECK(s.submit(5, nullptr, 10, 1, 0, 0.3, &id[3]) == kSchedInval);
  CHECK(s.submit(0, nullptr, 10, 100, 0, 0.4, &id[3]) == kSchedOk);
  CHECK(s.submit(0, nullptr, 10, 100, 0, 0.4, &id[4]) == kSchedOk);
  CHECK(s.submit(0, nullptr, 10, 100, 0, 0.4, &id[5]) == kSchedAgain);  // queue of 5 is full
  auto all = [](Request&) { return true; };
  // two slots: the first two are admitted (800 of 1000 bytes)
  std::vector<Request*> a1 = s.admit(1.0, all);
  CHECK(a1.size() == 2 && a1[0]->id == id[0] && a1[1]->id == id[1]);
  CHECK(s.used() == 800 && s.inflight() == 2);
  // no slot: nothing more
  CHECK(s.admit(1.1, all).empty());
  s.complete(id[0], kReqDone, 2.0, 7, 3);
  // a slot is free and request 3 (100 bytes) would fit, but request 2 (700
  // bytes) does not fit 1000 - 400 and admission is FIFO: nothing

  CHECK(s.admit(2.0, all).empty());
  s.complete(id[1], kReqDone, 3.0, 8, 3);
  std::vector<Request*> a2 = s.admit(3.0, all);
  CHECK(a2.size() == 2 && a2[0]->id == id[2] && a2[1]->id == id[3]);
  // cancel: queued -> cancelled; running -> again; unknown -> not found
  CHECK(s.cancel(id[4], 3.5) == kSchedOk && s.find(id[4])->state == kSchedCancelled);
  CHECK(s.cancel(id[2], 3.5) == kSchedAgain);
  CHECK(s.cancel(999, 3.5) == kSchedNotFound);
  // a failed reservation holds admission back
  s.complete(id[2], kReqDone, 4.0, 1, 2);
  uint64_t late = 0;
  CHECK(s.submit(1, nullptr, 10, 10, 0, 4.0, &late) == kSchedOk);
  CHECK(s.admit(4.0, [](Request&) { return false; }).empty());
  CHECK(s.find(late)->state == kReqQueued);
  s.complete(id[3], -3, 5.0, -1, 0);  // a failed request frees its slot and budget
  CHECK(s.stats().failed == 1);
  CHECK(s.admit(5.0, all).size() == 1);
  s.complete(late, kReqDone, 6.0, 0, 1);
  CHECK(s.used() == 0 && s.inflight() == 0);
  const SchedStats& st = s.stats();
  CHECK(st.completed == 4 && st.rejected == 2 && st.cancelled == 1 && st.keys_completed == 40);
  // latencies 2.0, 2.9, 3.8, 2.0 -> sorted 2.0 2.0 2.9 3.8
  CHECK(std::abs(Scheduler::percentile(st.latencies, 0.5) - 2.45) < 1e-12);
  CHECK(std::abs(Scheduler::percentile(st.latencies, 1.0) - 3.8) < 1e-12);
  CHECK(Scheduler::percentile({}, 0.5) == 0.0);
}

int main() {
  range_alloc();
  scheduler();
  if (failures) {
    std::fprintf(stderr, "%d checks failed\n", failures);
    return 1;
  }
  std::puts("sched checks passed");
  return 0;
}
