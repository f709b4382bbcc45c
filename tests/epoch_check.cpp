// Host checks of the look-back tag rule and of what a server lane may clear
// when the tags wrap (no GPU).  Uses the library's own rule (ksort_epoch.h).
//
// 1. Over many spans, with random tiles publishing words in every pass, a
//    reader of pass s never accepts a word that pass s did not write when the
//    words are cleared exactly where epoch_wraps_before() says; without those
//    clears a stale word is accepted.
// 2. A lane model: requests in flight keep their segments in the stage lists
//    (a ring of three counters, as the kernels keep them).  Clearing only the
//    tags at the wrap lets every request complete; clearing the counters as
//    well (what a full reset does) loses the segments listed for the next
//    pass, and their requests never complete.
// 3. kernel_stage() keeps the counter ring and the list parity of the 64-bit
//    pass number, also across its own wrap and beyond 2^31 passes.
#include <cstdint>
#include <cstdio>
#include <random>
#include <vector>

#include "ksort_epoch.h"

using namespace ksort;

static int failures = 0;
#define CHECK(c)                                                          \
  do {                                                                    \
    if (!(c)) {                                                           \
      std::fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #c); \
      ++failures;                                                         \
    }                                                                     \
  } while (0)

// Word layout of the kernels: count in bits 0..39, flag in 40..41, tag in 42..63.
static uint64_t word(uint32_t tag, uint64_t flag, uint64_t count) { return ((uint64_t)tag << 42) | (flag << 40) | count; }
static bool accepted(uint64_t w, uint32_t tag) { return (uint32_t)(w >> 42) == tag && ((w >> 40) & 3) != 0; }

// Returns the number of stale words a reader accepted.
static long replay_words(int64_t span, int64_t passes, bool clear_at_wrap, unsigned seed) {
  std::mt19937_64 rng(seed);
  const int nwords = 64;
  std::vector<uint64_t> w(nwords, 0);
  std::vector<int64_t> written_in(nwords, -1);
  long stale = 0;
  for (int64_t s = 0; s < passes; ++s) {
    if (clear_at_wrap && epoch_wraps_before(s, span)) {
      for (auto& x : w) x = 0;
    }
    const uint32_t tag = epoch_of(s, span);
    CHECK(tag >= 1 && tag <= (uint32_t)kEpochSpanMax);
    // some tiles of this pass publish (a random prefix of the tile map: a
    // pass uses tickets 0 .. ntiles-1)
    const int ntiles = (int)(rng() % nwords);
    const int published = ntiles ? (int)(rng() % (ntiles + 1)) : 0;
    for (int j = 0; j < published; ++j) {
      w[j] = word(tag, 1 + (rng() & 1), rng() & 0xffff);
      written_in[j] = s;
    }
    // a tile of this pass reads its predecessors' words
    for (int j = 0; j < ntiles; ++j)
      if (accepted(w[j], tag) && written_in[j] != s) ++stale;
  }
  return stale;
}

// Ring of three stage counters holding how many segments each stage lists;
// every request in flight keeps one segment per pass until its last pass.
struct LaneModel {
  int64_t ctr[3] = {0, 0, 0};
  std::vector<int> left;  // passes left per request in flight
};

static int run_lane(int64_t span, int64_t passes, bool full_reset) {
  LaneModel L;
  std::mt19937 rng(7);
  int completed = 0, admitted = 0;
  for (int64_t s = 0; s < passes; ++s) {
    if (epoch_wraps_before(s, span) && full_reset) {
      for (auto& c : L.ctr) c = 0;  // a full reset also clears the counters
    }
    // admission into the current stage's list
    if (L.left.size() < 8) {
      L.left.push_back(3 + (int)(rng() % 20));
      L.ctr[s % 3] += 1;
      ++admitted;
    }
    // the pass runs the segments listed for it; each request lists one for
    // the next pass unless this was its last
    const int64_t listed = L.ctr[s % 3];
    L.ctr[(s + 2) % 3] = 0;  // the kernel clears the counter of the stage after next
    std::vector<int> still;
    int64_t run = 0;
    for (int r : L.left) {
      if (run < listed) {
        ++run;
        if (--r == 0) {
          ++completed;
          continue;
        }
        L.ctr[(s + 1) % 3] += 1;
      }
      still.push_back(r);
    }
    L.left.swap(still);
  }
  // drain without admissions
  for (int64_t s = passes; s < passes + 64; ++s) {
    const int64_t listed = L.ctr[s % 3];
    L.ctr[(s + 2) % 3] = 0;
    std::vector<int> still;
    int64_t run = 0;
    for (int r : L.left) {
      if (run < listed) {
        ++run;
        if (--r == 0) {
          ++completed;
          continue;
        }
        L.ctr[(s + 1) % 3] += 1;
      }
      still.push_back(r);
    }
    L.left.swap(still);
  }
  return admitted - completed;  // requests that never complete
}

int main() {
  // 1. the tag rule
  for (int64_t span : {2, 3, 5, 17, 1000}) {
    for (unsigned seed = 1; seed <= 4; ++seed) {
      CHECK(replay_words(span, 12 * span + 7, true, seed) == 0);
    }
    long stale = 0;
    for (unsigned seed = 1; seed <= 4; ++seed) stale += replay_words(span, 12 * span + 7, false, seed);
    CHECK(stale > 0);  // the clears are needed
  }
  CHECK(epoch_of(kEpochSpanMax - 1, kEpochSpanMax) == (uint32_t)kEpochSpanMax);
  CHECK(epoch_of(kEpochSpanMax, kEpochSpanMax) == 1u);
  CHECK(!epoch_wraps_before(0, 3) && epoch_wraps_before(3, 3) && !epoch_wraps_before(4, 3));
  CHECK(epoch_wraps_before(3 * kEpochSpanMax, kEpochSpanMax));
  // 2. what the wrap may clear
  for (int64_t span : {2, 3, 7}) {
    CHECK(run_lane(span, 200, false) == 0);  // tags only: everything completes
    CHECK(run_lane(span, 200, true) > 0);    // counters too: requests are lost
  }
  // 3. the lane's pass number
  for (int64_t s : {int64_t(0), int64_t(5), kStageRing - 1, kStageRing, kStageRing + 1, (int64_t(1) << 31) + 3,
                    int64_t(7) * kStageRing + 11, int64_t(1) << 40}) {
    const int32_t k = kernel_stage(s);
    CHECK(k >= 0 && (int64_t)k < kStageRing);
    CHECK(k % 3 == s % 3 && (k & 1) == (s & 1));
    CHECK((int64_t)k + 2 < ((int64_t)1 << 31));  // stage + 1 and + 2 stay in 32 bits
  }
  // consecutive passes across the ring's wrap keep consecutive ring slots
  for (int64_t s = kStageRing - 4; s < kStageRing + 4; ++s) {
    CHECK((kernel_stage(s) + 1) % 3 == kernel_stage(s + 1) % 3);
    CHECK((kernel_stage(s) & 1) != (kernel_stage(s + 1) & 1));
  }
  if (failures) {
    std::fprintf(stderr, "%d checks failed\n", failures);
    return 1;
  }
  std::printf("epoch checks passed\n");
  return 0;
}
