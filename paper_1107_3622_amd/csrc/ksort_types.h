// Descriptor and argument types shared by the K-sort kernels and the host
// driver (no device code).
#pragma once

#include <stdint.h>

namespace ksort {

// A segment of one stage (48 bytes).  Live segments (len > cutoff) carry
// first_tile; finish segments (1 <= len <= cutoff) do not use it.  Every
// segment carries the two buffers of its array, so a tile or a finish task
// needs one descriptor load before it can load keys.
struct Seg {
  int64_t left;        // index of the segment's first key in its buffers
  int64_t len;         // number of keys
  void* data;          // the caller's array; final keys are written here
  void* scratch;       // ping-pong partner with the same extent
  int32_t root;        // >= 0: the segment is a whole input array, index of its pivot slot
  int32_t buf;         // request slot (completion accounting of the server)
  int32_t parity;      // 0: keys are in data, 1: in scratch
  int32_t first_tile;  // first partition ticket of the segment's tiles
};

struct BufPair {
  void* data;
  void* scratch;
};

// Per-stage counters; stage s appends its children to ctr[(s + 1) % 3] and
// clears ctr[(s + 2) % 3] for the stage after next.
struct StageCtr {
  int32_t nseg;      // live segments appended
  int32_t ntiles;    // partition tickets reserved
  int32_t nfin;      // finish segments appended
  int32_t ticket;    // work tickets claimed
  int32_t carry;     // finish tasks carried over from the stage before (upper half of the list)
  int32_t pad[3];
};

struct Flags {
  int32_t last_active;  // highest stage index that has work
  int32_t err;          // invalid input segment seen by the init kernel
  int32_t overflow;     // a device check failed: 1-3 capacity or count, 4 a look-back wait timed out
  int32_t diag_stage;   // code 4: the pass whose wait timed out (first failure only)
  int32_t diag_tile;    // code 4: ticket index of the waiting tile in that pass's tile map
  int32_t diag_pred;    // code 4: ticket index of the predecessor it waited for
  uint64_t diag_word;   // code 4: that predecessor's look-back word when the wait gave up
};

struct StageArgs {
  StageCtr* ctr;          // ring of 3
  Seg* live[2];           // live lists by stage parity
  int32_t* tilemap[2];    // partition ticket -> live slot, by stage parity
  Seg* fin[2];            // finish lists by stage parity
  uint64_t* status;       // look-back words, one per partition ticket
  int64_t* pivot_out;     // per root (nullable)
  int32_t* pending;       // per request slot: outstanding segments (nullable)
  int32_t* done_stage;    // per request slot: stage at which pending hit 0 (nullable)
  Flags* flags;
  int64_t* stage_keys;    // [cap_stats][2]: keys partitioned, keys finished (nullable)
  int32_t cap_live, cap_tiles, cap_fin, cap_stats;
  int32_t stage;
  uint32_t epoch;         // tag of this stage's look-back words (22 bits, never 0)
  int32_t cutoff;         // sides of at most this many keys go to finish work
  int32_t emit_children;  // 0: one level only (no recursion)
  int32_t pivot_relative; // pivot reported as i - left (1) or as i (0)
  int32_t fin_run;        // finish tasks a stage with partition tiles runs; the rest wait a stage
  int32_t fin_half;       // finish lists: children below this index, carried tasks from it up
  uint32_t spin_limit;    // polls of a look-back wait before the pass gives up (flag code 4)
  int32_t fixed_first;    // 1: workgroup b takes ticket b first (no counter); 0: every ticket from the counter
};

// Arguments of the set-up kernel that turns input arrays (or, for a single
// level, caller-given segments) into the lists of one stage.
struct InitArgs {
  StageArgs sa;              // lists, counters and flags of the run
  BufPair pair;              // the arrays' buffers
  int32_t buf;               // request slot of these arrays
  int32_t root_base;         // pivot slot of array 0
  int64_t n;                 // extent of the caller's array
  const int64_t* offsets;    // nseg + 1 array offsets (sort modes), or null
  const int64_t* seg_left;   // segment starts (single-level mode)
  const int64_t* seg_len;    // segment lengths (single-level mode)
  int64_t nseg;
  int32_t level_mode;        // 1: every segment gets one partition, keys read from scratch
  int32_t tile;              // keys per partition tile
};

}  // namespace ksort
