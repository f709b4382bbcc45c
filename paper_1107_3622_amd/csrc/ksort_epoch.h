// Epoch tags of the look-back words (pure C++, no HIP, so the rule can be
// checked on the host on its own).
//
// A partition tile publishes its count in a 64-bit word tagged with the
// epoch of its level pass; a reader accepts a word only if the tag equals its
// own pass's epoch.  Words are therefore never cleared between passes: a word
// left by an earlier pass carries another tag.  Tags have 22 bits and 0 means
// "never written", so a run of passes 0, 1, 2, ... uses the tags
//     epoch(s) = (s mod span) + 1,   span <= 2^22 - 1,
// and before pass s with s > 0 and s mod span == 0 the words must be cleared:
// only then could a word of pass s - span (same tag) still be read as one of
// pass s.  Clearing touches the look-back words and nothing else; counters,
// lists and flags of work in flight are left alone.
#pragma once

#include <stdint.h>
#include <stdlib.h>

namespace ksort {

constexpr int64_t kEpochSpanMax = (1 << 22) - 1;  // tags 1 .. 2^22 - 1

inline uint32_t epoch_of(int64_t stage, int64_t span) { return (uint32_t)(stage % span) + 1u; }

// True when the look-back words must be cleared before pass `stage`.
inline bool epoch_wraps_before(int64_t stage, int64_t span) { return stage > 0 && stage % span == 0; }

// A server lane counts its passes in 64 bits and runs pass s as kernel pass
// s mod kStageRing: the ring is a multiple of 6, so the kernels' counter ring
// (stage mod 3) and list parity (stage mod 2) go on unchanged across its
// wrap, and it fits the kernels' 32-bit stage.  Look-back tags come from s.
constexpr int64_t kStageRing = 6ll << 28;
inline int32_t kernel_stage(int64_t s) { return (int32_t)(s % kStageRing); }

// The span used by a run: 2^22 - 1, or KSORT_EPOCH_SPAN (a decimal count in
// [2, 2^22 - 1]) when it is set, so that tests can reach the wrap in a few
// passes.  Read when a run or a server lane starts and kept for its duration.
inline int64_t epoch_span_setting() {
  const char* s = getenv("KSORT_EPOCH_SPAN");
  if (!s || !*s) return kEpochSpanMax;
  char* end = nullptr;
  const long long v = strtoll(s, &end, 10);
  if (*end != '\0' || v < 2 || v > kEpochSpanMax) return kEpochSpanMax;
  return (int64_t)v;
}

}  // namespace ksort
