// K-sort device kernels for gfx950 (CDNA4, wave64).
//
// The paper's method (arXiv 1107.3622, Section 1.1) partitions a[left..right]
// around key = a[left]: keys for which `key <= x` is false go left of the key,
// the others right, and both sides are then treated the same way.  Step-4
// leaves the key at i = left + (number of keys smaller than it); Steps 5-6
// recurse on [left, i-1] and [i+1, right]; a side with one key is final
// (Section 1.2 note).
//
// Every level of that recursion is one data-parallel pass over all live
// segments at once (the stage kernel), with two kinds of work:
//   * partition tiles: each live segment is cut into tiles of BLOCK*ITEMS
//     keys.  A tile classifies its keys against the segment's key with one
//     compare each, counts them with wave ballots and popcounts, scans the
//     per-wave counts in LDS, obtains the count of smaller keys in the
//     segment's earlier tiles by decoupled look-back, and scatters its keys
//     from registers into the ping-pong buffer: smaller keys fill [left, i-1]
//     upward, the others fill [i+1, right] downward, so i need not be known
//     in advance.  The segment's last tile knows i, writes the key to its
//     final place in the caller's array and emits the two sides.  When the
//     segment had a single tile, the same workgroup may go on with one side
//     of CUT+1 .. BLOCK*ITEMS keys in the same pass (a chain of one-tile
//     segments), in passes where that cannot end the pass late.
//   * finish tasks: a segment of at most CUT keys is loaded into LDS once
//     and sorted there by the same rule: the workgroup partitions the top of
//     the recursion, then its waves take sub-segments from an LDS queue and
//     partition them with wave ballots between two LDS buffers; a
//     sub-segment of at most kLeaf keys is placed by rank.  Every key is
//     written straight to its final place.
// Both kinds of work come from one ticket counter per stage, finish tasks
// first, so a persistent grid drains the stage without host involvement; a
// stage with no partition tiles hands out finish tickets in batches.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ksort_types.h"

namespace ksort {

constexpr int kWave = 64;

// ---------------------------------------------------------------------------
// small helpers

// Pointers into device memory.  Descriptors carry generic pointers; casting
// them to the global address space, with a wave-uniform base and 32-bit byte
// offsets, lets the compiler use global loads and stores with a scalar base
// register instead of flat accesses with 64-bit per-lane addresses.
#define KS_GLOBAL __attribute__((address_space(1)))

// Compiler-level helpers written as inline assembly.  A build may define
// them beforehand (the host test build of the kernels does).
//   KS_OPAQUE(x)  : x passes through an empty asm in a vector register, so the
//                   optimizer cannot recompute or hoist what it depends on
//   KS_LDS_WAIT() : wait until this wave's LDS operations have completed
//   KS_MEM_FENCE(): a compiler-only memory barrier
//   KS_WAVE_STEP(): marks a point where the code relies on the lanes of a wave
//                   executing in step (a lane reads what other lanes of its
//                   wave wrote to LDS just before); no instruction on the
//                   hardware, where a wave always executes in step
#ifndef KS_OPAQUE
#define KS_OPAQUE(x) asm volatile("" : "+v"(x))
#endif
#ifndef KS_LDS_WAIT
#define KS_LDS_WAIT() asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory")
#endif
#ifndef KS_MEM_FENCE
#define KS_MEM_FENCE() asm volatile("" ::: "memory")
#endif
#ifndef KS_WAVE_STEP
#define KS_WAVE_STEP()
#endif

template <typename T>
__device__ __forceinline__ T gld(const void* base, uint32_t byte_off) {
  return *(const KS_GLOBAL T*)((const KS_GLOBAL char*)base + byte_off);
}
template <typename T>
__device__ __forceinline__ void gst(void* base, uint32_t byte_off, T v) {
  *(KS_GLOBAL T*)((KS_GLOBAL char*)base + byte_off) = v;
}

// 16-byte vectors of keys with only the keys' own alignment (a tile starts
// wherever its segment does).  A build may define KeyVec beforehand (the
// host test build does, with a plain struct).
#ifndef KS_KEY_VEC_DEFINED
template <typename T>
struct KeyVec;
template <>
struct KeyVec<float> {
  typedef float type __attribute__((ext_vector_type(4), aligned(4)));
};
template <>
struct KeyVec<double> {
  typedef double type __attribute__((ext_vector_type(2), aligned(8)));
};
#endif
// Keys per tile load: four FP32 keys (16 bytes) when the items per thread
// come in whole groups of four, else one (KSORT_VEC_LOADS=0: always one).
// Measured: 2^29 FP32 47.0 against 48.5 ms, 7e6 FP32 0.903 against 0.912.
// FP64 keeps one key per load: two per load gained 0.5 % at 2^28 and took
// the 28-key variant from 125 to 138 VGPRs, past the 128 that four waves
// per SIMD allow (7e6: 1.38 against 1.00 ms).
#ifndef KSORT_VEC_LOADS
#define KSORT_VEC_LOADS 1
#endif
template <typename T, int ITEMS>
constexpr int vec_keys() {
  return KSORT_VEC_LOADS && sizeof(T) == 4 && ITEMS % 4 == 0 ? 4 : 1;
}

__device__ __forceinline__ int lane_id() { return threadIdx.x & (kWave - 1); }

__device__ __forceinline__ int mbcnt(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0));
}

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ int64_t uniform64(int64_t v) {
  uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

template <typename P>
__device__ __forceinline__ P* uniform_ptr(P* p) {
  return (P*)uniform64((int64_t)(uintptr_t)p);
}

template <typename I>
__device__ __forceinline__ I ld_agent(I* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename I>
__device__ __forceinline__ void st_agent(I* p, I v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename I>
__device__ __forceinline__ I add_agent(I* p, I v) {
  return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename I>
__device__ __forceinline__ I ld_group(I* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Inclusive prefix sum across the 64 lanes of a wave, in registers: row
// shifts by 1, 2, 4 and 8 give every lane the prefix within its 16-lane row;
// the row broadcasts of lanes 15 and 31 then add the totals of the rows
// before it.  Every lane of the wave must be active.
__device__ __forceinline__ int wave_inclusive_scan(int v) {
  v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, false);  // row_shr:1
  v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, false);  // row_shr:2
  v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, false);  // row_shr:4
  v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, false);  // row_shr:8
  v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xa, 0xf, false);  // row_bcast:15 into rows 1 and 3
  v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xc, 0xf, false);  // row_bcast:31 into rows 2 and 3
  return v;
}

// Sum of v over the 64 lanes of a wave (the last lane of the inclusive
// scan), returned in every lane.  Every lane of the wave must be active.
__device__ __forceinline__ int wave_sum(int v) {
  return __builtin_amdgcn_readlane(wave_inclusive_scan(v), kWave - 1);
}

// The value v holds in lane j (j wave-uniform).
__device__ __forceinline__ int64_t lane_read64(int64_t v, int j) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(uint64_t)v, j);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)v >> 32), j);
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

// The value v holds in lane j (j wave-uniform).
__device__ __forceinline__ float lane_read(float v, int j) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), j));
}
__device__ __forceinline__ double lane_read(double v, int j) {
  const uint64_t u = (uint64_t)__double_as_longlong(v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, j);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), j);
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// Look-back word: count in bits 0..39, flag in 40..41, epoch in 42..63.
constexpr uint64_t kFlagAgg = 1;   // tile's own count of smaller keys
constexpr uint64_t kFlagPre = 2;   // count over the segment up to and including the tile
__device__ __forceinline__ uint64_t status_word(uint32_t epoch, uint64_t flag, uint64_t count) {
  return ((uint64_t)epoch << 42) | (flag << 40) | count;
}

// ---------------------------------------------------------------------------
// work items

constexpr int kTaskUnclaimed = -1;  // the block has not claimed its next ticket yet
constexpr int kTaskNone = 0;
constexpr int kTaskTile = 1;
constexpr int kTaskFinish = 2;

struct Task {
  Seg seg;
  int32_t kind;
  int32_t t;  // partition tiles: index into the stage's tile map (look-back slot)
  int32_t bnext, bend;  // tickets [bnext, bend) claimed with this one and not yet taken
};

// Finish tickets claimed at once in a stage without partition tiles.
constexpr int32_t kFinBatch = 32;

__device__ __forceinline__ void load_seg(Seg* d, const KS_GLOBAL Seg* s) {
  d->left = s->left;
  d->len = s->len;
  d->data = s->data;
  d->scratch = s->scratch;
  d->root = s->root;
  d->buf = s->buf;
  d->parity = s->parity;
  d->first_tile = s->first_tile;
}
__device__ __forceinline__ void store_seg(KS_GLOBAL Seg* d, const Seg& s) {
  d->left = s.left;
  d->len = s.len;
  d->data = s.data;
  d->scratch = s.scratch;
  d->root = s.root;
  d->buf = s.buf;
  d->parity = s.parity;
  d->first_tile = s.first_tile;
}

// What a stage holds, as every workgroup reads it at the start: partition
// tiles, work tickets (finish tasks run in this stage, then tiles) and the
// number of finish tasks carried over from the stage before.  Carried tasks
// (upper half of the finish list) take the first tickets, so a task is
// carried at most as long as newer ones keep the grid busy.
struct Counts {
  int32_t ntiles, nwork, ncar;
};

// Slot in the finish list of this stage's finish task number t.
__device__ __forceinline__ int32_t fin_slot(const StageArgs& a, const Counts& cn, int32_t t) {
  return t < cn.ncar ? a.fin_half + t : t - cn.ncar;
}

// Tickets handed out by the stage's counter start at this value: the grid
// size when every workgroup took its first ticket without the counter.
__device__ __forceinline__ int32_t ticket_base(const StageArgs& a) {
  return a.fixed_first ? (int32_t)gridDim.x : 0;
}

// Claims the next ticket of the stage and resolves it to a work item
// (executed by one thread; the result goes to LDS for the block).
//
// A partition tile waits in its look-back for tiles with lower tickets, so
// the holder of every lower ticket must be a workgroup that is running.
// With tickets from the counter that holds by construction: a ticket is
// claimed by a running workgroup, and the holder of the lowest unfinished
// ticket never waits.  With fixed first tickets (a.fixed_first), workgroup b
// takes ticket b without an atomic (512 simultaneous claims on one counter
// cost several microseconds per stage) and later tickets come from the
// counter offset by the grid size; then every workgroup of the grid must be
// dispatched while earlier ones wait, which holds when nothing else occupies
// the device: the grid never exceeds what the device holds at once, and the
// host orders all stage-kernel launches of a device one after another.  A
// kernel of other code that keeps part of the device busy delays the
// dispatch of the remaining workgroups for as long as it or its successors
// hold those slots, and tiles with counter tickets wait that long in their
// look-back.  Where request producers run kernels at the same time by design
// (the server), every ticket comes from the counter.
__device__ __forceinline__ void fetch_task(const StageArgs& a, StageCtr* cur, const Counts& cn, Task* out,
                                           int32_t first = -1) {
  const int par = a.stage & 1;
  int32_t t;
  if (first >= 0) {
    t = first;
    out->bnext = out->bend = 0;
  } else if (out->bnext < out->bend) {
    t = out->bnext++;
  } else {
    // In a stage without partition tiles nobody waits on a ticket's holder,
    // so finish tickets are claimed in batches: one counter shared by the
    // whole grid serves only a limited number of claims per microsecond.
    // The batch shrinks as the tickets run out, to keep the stage's end even.
    int32_t b = 1;
    if (cn.ntiles == 0) {
      const int32_t rest = cn.nwork - (ld_agent(&cur->ticket) + ticket_base(a));
      b = min(kFinBatch, max(1, rest / (4 * (int32_t)gridDim.x)));
    }
    t = add_agent(&cur->ticket, b) + ticket_base(a);
    out->bnext = t + 1;
    out->bend = t + b;
  }
  out->t = t;
  // Finish tasks take the first tickets: they never wait on anyone and take
  // longer than a tile, so starting them first keeps them off the end of the
  // stage.  Partition tiles follow in segment order (the look-back relies on
  // a tile's predecessors holding lower tickets).
  const int32_t nfin = cn.nwork - cn.ntiles;
  if (t < nfin) {
    load_seg(&out->seg, (const KS_GLOBAL Seg*)a.fin[par] + fin_slot(a, cn, t));
    out->kind = kTaskFinish;
  } else if (t < cn.nwork) {
    const int32_t tt = t - nfin;
    const int32_t slot = ((const KS_GLOBAL int32_t*)a.tilemap[par])[tt];
    load_seg(&out->seg, (const KS_GLOBAL Seg*)a.live[par] + slot);
    out->kind = kTaskTile;
    out->t = tt;
  } else {
    out->kind = kTaskNone;
  }
}

// Finish work claims its successor early, hiding the claim behind the sort,
// but only while finish tickets remain: a partition tile is claimed only when
// the block is free to load it, because every later tile of its segment waits
// for its count in the look-back.
__device__ __forceinline__ void claim_early(const StageArgs& a, StageCtr* cur, const Counts& cn, Task* out) {
  if (out->bnext < out->bend || ld_agent(&cur->ticket) + ticket_base(a) < cn.nwork - cn.ntiles)
    fetch_task(a, cur, cn, out);
  else
    out->kind = kTaskUnclaimed;
}

// A work item read from LDS, with every field wave-uniform.
struct TaskU {
  int64_t left, len;
  void* data;
  void* scratch;
  int32_t root, buf, parity, first_tile, kind, t;
};

__device__ __forceinline__ TaskU read_task(const Task* tk) {
  TaskU u;
  u.left = uniform64(tk->seg.left);
  u.len = uniform64(tk->seg.len);
  u.data = uniform_ptr(tk->seg.data);
  u.scratch = uniform_ptr(tk->seg.scratch);
  u.root = uniform(tk->seg.root);
  u.buf = uniform(tk->seg.buf);
  u.parity = uniform(tk->seg.parity);
  u.first_tile = uniform(tk->seg.first_tile);
  u.kind = uniform(tk->kind);
  u.t = uniform(tk->t);
  return u;
}

// ---------------------------------------------------------------------------
// shared memory layouts

template <typename T, int BLOCK, int ITEMS>
struct PartSmem {
  static constexpr int NW = BLOCK / kWave;
  int32_t off_lt[ITEMS * NW];
  int32_t off_ge[ITEMS * NW];
  int64_t xlt;
  int32_t tot_lt, tot_ge;
  int32_t em_slot[2], em_first[2], em_nt[2];
  int64_t inl_left, inl_len;  // the child this workgroup partitions next, if inl_c >= 0
  int32_t inl_c;
  int32_t inl_listed;         // sides the last segment put on the lists
};

// A chain of one-tile partitions within one pass puts at most this many sides
// on the next pass's lists (the finish lists hold that many per live segment).
constexpr int kChainLists = 4;

// Sub-segments of the wave queue with at most kLeaf keys are placed by rank
// (one, two or four keys per lane) instead of being partitioned further.
#ifndef KSORT_LEAF
#define KSORT_LEAF 128
#endif
constexpr int kLeaf = KSORT_LEAF;
static_assert(kLeaf == 64 || kLeaf == 128 || kLeaf == 256, "one, two or four keys per lane");

template <typename T, int BLOCK, int CUT>
struct FinSmem {
  static constexpr int NW = BLOCK / kWave;
  static constexpr int QCAP = CUT + NW + 2;
  T buf[2][CUT];       // ping-pong buffers of the segment
  uint32_t q[QCAP];    // sub-segment queue; 0 = slot not yet written
  int32_t q_head, q_tail, outstanding;
  int32_t bcnt[(CUT / BLOCK) * NW];  // workgroup partition: per-(item, wave) counts
  int32_t bc;                        // workgroup partition: smaller keys in the sub-segment
  int32_t tie[NW][kLeaf];            // per wave: placement of equal keys in a leaf
};

template <typename T, int BLOCK, int ITEMS, int CUT>
union StageSmem {
  PartSmem<T, BLOCK, ITEMS> p;
  FinSmem<T, BLOCK, CUT> f;
};

// ---------------------------------------------------------------------------
// decoupled look-back: the number of smaller keys in tiles first_tile .. t-1
// of the segment.  Executed by one whole wave.  Each round examines
// kLookBack*64 predecessors (lane j, slot r watches tile t-1-j-64r, so slot 0
// holds the nearest 64), which lets the front of published prefixes advance
// that many tiles per memory round trip.

constexpr int kLookBack = 4;

// Returns -1 if a predecessor has not published after a.spin_limit polls,
// or once the pass has failed elsewhere (the wait is bounded, so a lost or
// never-claimed predecessor ends the pass with an error instead of holding
// the device).
__device__ __forceinline__ int64_t look_back(const StageArgs& a, int32_t t, int32_t first_tile) {
  const int lane = lane_id();
  int64_t excl = 0;
  int32_t base = t - 1;
  uint32_t polls = 0;
  for (;;) {
    uint64_t w[kLookBack];
    bool in_seg[kLookBack];
#pragma unroll
    for (int r = 0; r < kLookBack; ++r) {
      const int32_t j = base - lane - kWave * r;
      in_seg[r] = j >= first_tile;
      w[r] = in_seg[r] ? ld_agent(a.status + j) : 0;
    }
    // wait (per lane) until every watched predecessor has published
    bool timed_out = false;
    for (;;) {
      bool ready = true;
#pragma unroll
      for (int r = 0; r < kLookBack; ++r) {
        const bool ok = (uint32_t)(w[r] >> 42) == a.epoch && ((w[r] >> 40) & 3) != 0;
        ready = ready && (!in_seg[r] || ok);
      }
      if (ready) break;
      // gives up at the limit, or early once another wait of the pass has
      // failed (the pass is lost then, and every later tile of a segment
      // whose count never arrives would otherwise wait the full limit)
      if (++polls > a.spin_limit || ((polls & 255) == 0 && ld_agent(&a.flags->overflow) != 0)) {
        timed_out = true;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
#pragma unroll
      for (int r = 0; r < kLookBack; ++r) {
        const int32_t j = base - lane - kWave * r;
        const bool ok = (uint32_t)(w[r] >> 42) == a.epoch && ((w[r] >> 40) & 3) != 0;
        if (in_seg[r] && !ok) w[r] = ld_agent(a.status + j);
      }
    }
    if (__ballot(timed_out)) {
      // record the first predecessor still missing (the first failure of the
      // pass wins), then give up
      int32_t miss = -1;
      uint64_t mw = 0;
#pragma unroll
      for (int r = kLookBack - 1; r >= 0; --r) {
        const bool ok = (uint32_t)(w[r] >> 42) == a.epoch && ((w[r] >> 40) & 3) != 0;
        if (in_seg[r] && !ok) {
          miss = base - lane - kWave * r;
          mw = w[r];
        }
      }
      const uint64_t mm = __ballot(miss >= 0);
      if (mm && lane == __builtin_ctzll(mm) && atomicCAS(&a.flags->overflow, 0, 4) == 0) {
        a.flags->diag_stage = a.stage;
        a.flags->diag_tile = t;
        a.flags->diag_pred = miss;
        a.flags->diag_word = mw;
      }
      return -1;
    }
    // nearest predecessor with a full prefix: first slot with one, lowest
    // lane.  The predecessors nearer than it hold their own tile's count,
    // at most one tile's keys, so 64 of them sum in 32 bits.
#pragma unroll
    for (int r = 0; r < kLookBack; ++r) {
      const bool pre = in_seg[r] && ((w[r] >> 40) & 3) == kFlagPre;
      const uint64_t pre_mask = __ballot(pre);
      const int stop = pre_mask ? __builtin_ctzll(pre_mask) : kWave;
      const int64_t c = (int64_t)(w[r] & ((1ull << 40) - 1));
      excl += wave_sum(in_seg[r] && lane < stop ? (int)c : 0);
      if (pre_mask) return excl + lane_read64(c, stop);
    }
    base -= kWave * kLookBack;
  }
}

// ---------------------------------------------------------------------------
// The last tile of a live segment: Step-4 (the key to its final index i) and
// Steps 5-6 (the two sides become segments of the next stage).  All tiles of
// the segment have published their counts, hence have read their keys, so
// the key may be written into the caller's array even when that array is
// this stage's input.
// With `may_continue` (the segment had one tile), a side of cutoff+1 .. TILE
// keys is not listed: the workgroup partitions it next, in this pass (the
// larger one if both qualify).  Its keys were written by this workgroup, so
// they are visible to it after the barrier below.  *inl_c receives the side
// (0 left, 1 right) or -1, *inl_left and *inl_len its extent.
template <typename T, int TILE>
__device__ void emit_children(const StageArgs& a, int32_t* em_slot, int32_t* em_first, int32_t* em_nt,
                              const TaskU& tk, int64_t total_lt, T key, bool may_continue, int32_t* inl_c,
                              int64_t* inl_left, int64_t* inl_len, int32_t* inl_listed) {
  const int tid = threadIdx.x;
  const int par = a.stage & 1;
  const int64_t left = tk.left, len = tk.len;
  const int64_t i = left + total_lt;
  if (tid == 0) {
    *((KS_GLOBAL T*)tk.data + i) = key;
    if (tk.root >= 0 && a.pivot_out) a.pivot_out[tk.root] = a.pivot_relative ? total_lt : i;
    int nchild = 0, nlisted = 0;
    em_nt[0] = em_nt[1] = 0;
    *inl_c = -1;
    if (a.emit_children) {
      StageCtr* nx = a.ctr + ((a.stage + 1) % 3);
      const int npar = par ^ 1;
      const int64_t cl[2] = {left, i + 1};
      const int64_t cn[2] = {total_lt, len - 1 - total_lt};
      uint64_t live_keys = 0, fin_keys = 0;
      int cont = -1;
      if (may_continue) {
        for (int c = 0; c < 2; ++c)
          if (cn[c] > a.cutoff && cn[c] <= TILE && (cont < 0 || cn[c] > cn[cont])) cont = c;
      }
      if (cont >= 0) {
        *inl_c = cont;
        *inl_left = cl[cont];
        *inl_len = cn[cont];
        ++nchild;  // still outstanding for the completion count
        if (a.stage_keys && a.stage < a.cap_stats)
          atomicAdd((unsigned long long*)&a.stage_keys[2 * a.stage], (unsigned long long)cn[cont]);
      }
      for (int c = 0; c < 2; ++c) {
        if (c == cont) continue;
        Seg d;
        d.left = cl[c];
        d.len = cn[c];
        d.data = tk.data;
        d.scratch = tk.scratch;
        d.root = -1;
        d.buf = tk.buf;
        d.parity = tk.parity ^ 1;
        d.first_tile = 0;
        if (cn[c] > a.cutoff) {
          const int32_t nt = (int32_t)((cn[c] + TILE - 1) / TILE);
          const int32_t s = add_agent(&nx->nseg, 1);
          const int32_t f = add_agent(&nx->ntiles, nt);
          if (s >= a.cap_live || f + nt > a.cap_tiles) {
            st_agent(&a.flags->overflow, 1);
            continue;
          }
          d.first_tile = f;
          store_seg((KS_GLOBAL Seg*)a.live[npar] + s, d);
          em_slot[c] = s;
          em_first[c] = f;
          em_nt[c] = nt;
          ++nchild;
          ++nlisted;
          live_keys += (uint64_t)cn[c];
        } else if (cn[c] == 1 && tk.parity == 1) {
          // a one-key side written into the caller's array is already final
        } else if (cn[c] >= 1) {
          const int32_t f = add_agent(&nx->nfin, 1);
          if (f >= a.fin_half) {
            st_agent(&a.flags->overflow, 1);
            continue;
          }
          store_seg((KS_GLOBAL Seg*)a.fin[npar] + f, d);
          ++nchild;
          ++nlisted;
          fin_keys += (uint64_t)cn[c];
        }
      }
      if (nlisted > 0) atomicMax(&a.flags->last_active, a.stage + 1);
      *inl_listed = nlisted;
      if (a.stage_keys && a.stage + 1 < a.cap_stats) {
        if (live_keys) atomicAdd((unsigned long long*)&a.stage_keys[2 * (a.stage + 1)], live_keys);
        if (fin_keys) atomicAdd((unsigned long long*)&a.stage_keys[2 * (a.stage + 1) + 1], fin_keys);
      }
    }
    if (a.pending) {
      const int32_t old = add_agent(a.pending + tk.buf, nchild - 1);
      if (old + nchild - 1 == 0 && a.done_stage) st_agent(a.done_stage + tk.buf, a.stage);
    }
  }
  __syncthreads();
  // tile map of the live children: ticket -> live slot
  for (int c = 0; c < 2; ++c) {
    const int32_t nt = em_nt[c];
    if (nt > 0) {
      KS_GLOBAL int32_t* tm = (KS_GLOBAL int32_t*)a.tilemap[par ^ 1] + em_first[c];
      const int32_t s = em_slot[c];
      for (int j = tid; j < nt; j += blockDim.x) tm[j] = s;
    }
  }
}

// ---------------------------------------------------------------------------
// partition work: one tile of one live segment

// One partition tile.  Returns -1 after a failed consistency check (next is
// then kTaskNone), 1 if the workgroup continues with a child of this
// one-tile segment (sm.inl_*), else 0.  A continued child has no ticket
// (tk.t = -1): nothing waits on it and it publishes no look-back word.
template <typename T, int BLOCK, int ITEMS>
__device__ int partition_one(const StageArgs& a, const TaskU& tk, PartSmem<T, BLOCK, ITEMS>& sm, Task* next,
                             bool may_continue) {
  constexpr int NW = BLOCK / kWave;
  constexpr int TILE = BLOCK * ITEMS;
  constexpr int NC = ITEMS * NW;                 // per-(item, wave) counts
  constexpr int PER = (NC + kWave - 1) / kWave;  // counts scanned per lane
  static_assert(ITEMS <= 32, "per-thread masks are 32 bits");
  static_assert((int64_t)TILE * kWave < (1ll << 31), "the look-back sums 64 tile counts in 32 bits");
  int tid = threadIdx.x;
  // Opaque to the optimizer: keeps per-item offsets from being hoisted out of
  // the persistent loop, where they would hold dozens of registers for its
  // whole duration.
  KS_OPAQUE(tid);
  const int lane = tid & (kWave - 1), w = tid / kWave;

  const int32_t tidx = tk.t - tk.first_tile;
  const int64_t left = tk.left, len = tk.len;
  const int64_t o = (int64_t)tidx * TILE;
  const int32_t cnt = (int32_t)min((int64_t)TILE, len - o);
  const T* in = (const T*)(tk.parity ? tk.scratch : tk.data);
  T* out = (T*)(tk.parity ? tk.data : tk.scratch);
  const T key = gld<T>(in + left, 0);
  const T* src = in + left + o;

  // a1/a2: load the tile and classify each key against the segment's key.
  // Items come in groups of V keys that one 16-byte load brings in: item
  // k = g*V + c of thread tid is element g*BLOCK*V + tid*V + c (striped by
  // group, so each load instruction of a wave reads 1 KB contiguously).  Any
  // one-to-one map of (item, thread) to elements gives a valid partition,
  // since the counts are scanned in (item, wave) order and the scatter
  // follows the same order.  Group g of every lane lies below the uniform
  // base src + g*BLOCK*V; the lane offset tid*V*sizeof(T) is shared by all
  // groups, and "element exists" is tid*V + c < cnt - g*BLOCK*V (a uniform
  // bound), so no per-item index registers.  The segment's start has any
  // alignment: the 16-byte loads need only the keys' own alignment.
  constexpr int V = vec_keys<T, ITEMS>();
  const int tv = tid * V;
  T v[ITEMS];
  if (cnt == TILE) {
    if constexpr (V > 1) {
      typedef typename KeyVec<T>::type vec_t;
#pragma unroll
      for (int g = 0; g < ITEMS / V; ++g) {
        const vec_t q = gld<vec_t>(src + g * BLOCK * V, (uint32_t)tv * (uint32_t)sizeof(T));
#pragma unroll
        for (int c = 0; c < V; ++c) v[g * V + c] = q[c];
      }
    } else {
#pragma unroll
      for (int k = 0; k < ITEMS; ++k) v[k] = gld<T>(src + k * BLOCK, (uint32_t)tid * (uint32_t)sizeof(T));
    }
  } else {
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
      const int g = k / V, c = k % V;
      v[k] = (tv + c < cnt - g * BLOCK * V) ? gld<T>(src + g * BLOCK * V, (uint32_t)(tv + c) * (uint32_t)sizeof(T)) : T(0);
    }
  }
  // Per-item counts of the wave are gathered in one register (lane k: smaller
  // keys of item k, lane ITEMS+k: the others) and written with one store.
  // (The classification is recomputed, not stored, at scatter time: one
  // compare is cheaper than the registers a stored mask costs.)
  const bool not_key = !(tidx == 0 && tid == 0);  // element 0 of tile 0 is the key itself
  int wcnt = 0;
#pragma unroll
  for (int k = 0; k < ITEMS; ++k) {
    const bool valid = tv + k % V < cnt - (k / V) * BLOCK * V && (k > 0 || not_key);
    const bool lt = valid && !(key <= v[k]);
    const bool ge = valid && !lt;
    const uint64_t bl = __ballot(lt);
    const uint64_t bg = __ballot(ge);
    wcnt = lane == k ? __popcll(bl) : wcnt;
    wcnt = lane == ITEMS + k ? __popcll(bg) : wcnt;
  }
  if (lane < ITEMS)
    sm.off_lt[lane * NW + w] = wcnt;
  else if (lane < 2 * ITEMS)
    sm.off_ge[(lane - ITEMS) * NW + w] = wcnt;
  __syncthreads();

  // a3: exclusive scan of the per-(item, wave) counts in element order, then
  // the look-back for the smaller keys in the segment's earlier tiles.
  if (w == 0) {
    int cl[PER], cg[PER];
    int sl = 0, sg = 0;
#pragma unroll
    for (int j = 0; j < PER; ++j) {
      const int idx = lane * PER + j;
      cl[j] = idx < NC ? sm.off_lt[idx] : 0;
      cg[j] = idx < NC ? sm.off_ge[idx] : 0;
      sl += cl[j];
      sg += cg[j];
    }
    const int il = wave_inclusive_scan(sl);
    const int ig = wave_inclusive_scan(sg);
    int el = il - sl, eg = ig - sg;
#pragma unroll
    for (int j = 0; j < PER; ++j) {
      const int idx = lane * PER + j;
      if (idx < NC) {
        sm.off_lt[idx] = el;
        sm.off_ge[idx] = eg;
      }
      el += cl[j];
      eg += cg[j];
    }
    const int tot_lt = __builtin_amdgcn_readlane(il, kWave - 1);
    const int tot_ge = __builtin_amdgcn_readlane(ig, kWave - 1);
    if (lane == 0 && tk.t >= 0)
      st_agent(a.status + tk.t, status_word(a.epoch, tidx == 0 ? kFlagPre : kFlagAgg, (uint64_t)tot_lt));
    int64_t xlt = 0;
    if (tidx > 0) {
      xlt = look_back(a, tk.t, tk.first_tile);
      if (lane == 0 && xlt >= 0) st_agent(a.status + tk.t, status_word(a.epoch, kFlagPre, (uint64_t)(xlt + tot_lt)));
    }
    if (lane == 0) {
      sm.xlt = xlt;
      sm.tot_lt = tot_lt;
      sm.tot_ge = tot_ge;
    }
  }
  __syncthreads();

  // a4: scatter from registers.  Smaller keys fill [left, i-1] upward, the
  // others fill [i+1, right] downward.  The runs always lie inside the
  // segment; the check only guards the device against a corrupted count.
  const int64_t xlt = uniform64(sm.xlt);
  const int tot_lt = uniform(sm.tot_lt), tot_ge = uniform(sm.tot_ge);
  const int64_t xge = o - (tidx > 0 ? 1 : 0) - xlt;
  const int64_t right = left + len - 1;
  if (xlt < 0 || xge < 0 || xlt + tot_lt > len - 1 || xge + tot_ge > len - 1) {
    if (tid == 0) st_agent(&a.flags->overflow, xlt == -1 ? 4 : 2);
    if (tid == BLOCK - 1) next->kind = kTaskNone;
    return -1;
  }
  T* dlt = out + left + xlt;                  // first slot of this tile's smaller keys
  T* dge = out + (right - xge - tot_ge + 1);  // lowest slot of its other keys
  // Opaque copies: the compares below are recomputed rather than kept alive
  // since the counting loop (a compare costs less than the registers).
  T key2 = key;
  int tid2 = tid;
  KS_OPAQUE(key2);
  KS_OPAQUE(tid2);
  // this wave's offsets, one per lane as when they were counted
  const int woff = lane < ITEMS ? sm.off_lt[lane * NW + w] : lane < 2 * ITEMS ? sm.off_ge[(lane - ITEMS) * NW + w] : 0;
#pragma unroll
  for (int k = 0; k < ITEMS; ++k) {
    const bool valid = tid2 * V + k % V < cnt - (k / V) * BLOCK * V && (k > 0 || tidx != 0 || tid2 != 0);
    const bool lt = valid && !(key2 <= v[k]);
    const bool ge = valid && !lt;
    const int rl = mbcnt(__ballot(lt));
    const int rg = mbcnt(__ballot(ge));
    const int ol = __builtin_amdgcn_readlane(woff, k);
    const int og = __builtin_amdgcn_readlane(woff, ITEMS + k);
    if (lt) gst<T>(dlt, (uint32_t)((ol + rl) * sizeof(T)), v[k]);
    if (ge) gst<T>(dge, (uint32_t)((tot_ge - 1 - og - rg) * sizeof(T)), v[k]);
  }

  // a5/a6: the segment's last tile places the key and emits the two sides.
  if (o + cnt == len) {
    emit_children<T, TILE>(a, sm.em_slot, sm.em_first, sm.em_nt, tk, xlt + tot_lt, key, may_continue && len <= TILE,
                           &sm.inl_c, &sm.inl_left, &sm.inl_len, &sm.inl_listed);
    return uniform(sm.inl_c) >= 0 ? 1 : 0;
  }
  return 0;
}

// A partition tile, then, while its segment had one tile and a side of
// cutoff+1 .. TILE keys remains, that side's partition in the same pass:
// a chain of one-tile segments takes one pass instead of one per level.
// Every call is still Steps 1-4 on one segment with its first key.
template <typename T, int BLOCK, int ITEMS>
__device__ void partition_tile(const StageArgs& a, const TaskU& tk0, PartSmem<T, BLOCK, ITEMS>& sm, StageCtr* cur,
                               const Counts& cn, Task* next) {
  TaskU tk = tk0;
  int listed = 0;  // sides this chain has put on the lists
  // Chains run where they cannot end the pass late: in a pass with fewer
  // tiles than a quarter of the workgroups (the tail of the recursion, where
  // the next passes would otherwise hold little but these chains), or in a
  // pass of four or more rounds of tiles, whose end a chain of a few tiles
  // hardly moves.  In between, a chain started near the end of a pass of one
  // or two rounds would delay it (measured: +1.5 % at 7e6 when chains run
  // everywhere, -8 % with this rule; -6 % at 2^26 and -7 % at 2^28 either
  // way; at 1e6 this tail bound gave 0.46 ms against 0.51 with "fewer work
  // items than workgroups").
  const int32_t g = (int32_t)gridDim.x;
  const bool chain_pass = cn.ntiles < g / 4 || cn.ntiles >= 4 * g;
  for (;;) {
    // a step that continues lists at most one side, the last one at most two
    const int r = partition_one<T, BLOCK, ITEMS>(a, tk, sm, next, chain_pass && listed + 3 <= kChainLists);
    if (r < 0) return;
    if (r == 0) break;
    listed += uniform(sm.inl_listed);
    tk.left = uniform64(sm.inl_left);
    tk.len = uniform64(sm.inl_len);
    tk.parity ^= 1;
    tk.root = -1;
    tk.t = -1;
    tk.first_tile = -1;
    __syncthreads();  // sm is rewritten by the next partition
  }
  // the block is free: claim its next work item
  if (threadIdx.x == BLOCK - 1) fetch_task(a, cur, cn, next);
}

// ---------------------------------------------------------------------------
// finish work

constexpr int kSmall = kWave;  // sub-segments of at most this many keys finish in registers
constexpr int kBlockSide = 256;  // sides longer than this get a workgroup partition at the top

// Sorts in[0 .. L-1] (1 <= L <= 64) into out[0 .. L-1] with one wave, one key
// per lane, by placing every key at its rank: the number of keys smaller than
// it plus the number of equal keys before it.  For keys under a total order
// (no NaN, one sign of zero) this is the one ascending arrangement, so it is
// exactly what further K-sort levels would produce on the sub-segment, with
// no chain of dependent cross-lane steps.  The rank of the first key is the
// segment's Step-4 pivot offset (no key before it can tie), written to
// *pivot_slot when it is given.
// Order used to place keys by rank when a leaf holds a NaN (outside the
// bit-exact contract): numbers by value, every NaN after them.  Under it the
// ranks are still a permutation of 0 .. L-1, so the output stays a
// permutation of the input; without NaNs it is the plain `<`.
template <typename T>
__device__ __forceinline__ bool nan_last_less(T b, T v) {
  return b < v || (v != v && b == b);
}

template <typename T, typename In>
__device__ void wave_rank_sort(const In* in, T* out, int L, int64_t* pivot_slot, int64_t pivot_bias) {
  const int lane = lane_id();
  T v = lane < L ? (T)in[lane] : T(0);
  KS_OPAQUE(v);
  int rank = 0;
  int j = 0;
  if (__ballot(lane < L && v != v) == 0) {
    for (; j + 4 <= L; j += 4) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const T b = lane_read(v, j + u);
        rank += (b < v) | ((b <= v) & (j + u < lane));
      }
    }
    for (; j < L; ++j) {
      const T b = lane_read(v, j);
      rank += (b < v) | ((b <= v) & (j < lane));
    }
  } else {
    // a NaN is present: the same placement under nan_last_less, equal
    // (or both NaN) keys in lane order
    for (; j < L; ++j) {
      const T b = lane_read(v, j);
      rank += (int)nan_last_less(b, v) | ((int)!nan_last_less(v, b) & (int)(j < lane));
    }
  }
  if (lane < L) gst<T>(out, (uint32_t)(rank * sizeof(T)), v);
  if (pivot_slot && lane == 0) *pivot_slot = pivot_bias + rank;
}

// The same placement for a sub-segment held in LDS (2 <= L <= 64): every
// lane reads the keys it compares with as LDS broadcasts, two per read, and
// the main pass counts only the strictly smaller keys, one compare per pair.
// Those counts are the ranks exactly when the keys are distinct, which holds
// if and only if they sum to L(L-1)/2 (distinct ranks are 0 .. L-1, and a tie
// gives its keys the lower rank).  Otherwise the keys of a tie share a count
// c and must fill c, c+1, ...; they are equal bit for bit (total order), so
// any assignment among them gives the same array, and an LDS atomic on a
// per-wave counter for c hands them out.
//
// K keys per lane (lane + 64k) cover sub-segments of up to 64K keys.
template <typename T, int K>
__device__ void lds_rank_sort(const T* in, T* out, int L, int32_t* tie) {
  const int lane = lane_id();
  T v[K];
  int rank[K];
  bool nan = false;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    v[k] = lane + kWave * k < L ? in[lane + kWave * k] : T(0);
    rank[k] = 0;
    nan = nan || v[k] != v[k];
  }
  int j = 0;
  if (__ballot(nan) == 0) {
    for (; j + 8 <= L; j += 8) {
      T b[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) b[u] = in[j + u];
#pragma unroll
      for (int u = 0; u < 8; ++u)
#pragma unroll
        for (int k = 0; k < K; ++k) rank[k] += (int)(b[u] < v[k]);
    }
    for (; j < L; ++j) {
      const T b = in[j];
#pragma unroll
      for (int k = 0; k < K; ++k) rank[k] += (int)(b < v[k]);
    }
  } else {
    // a NaN is present (outside the bit-exact contract): count under
    // nan_last_less, so every NaN shares the count of all numbers and the
    // tie placement below gives them the last places
    for (; j < L; ++j) {
      const T b = in[j];
#pragma unroll
      for (int k = 0; k < K; ++k) rank[k] += (int)nan_last_less(b, v[k]);
    }
  }
  int sum = 0;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    if (lane + kWave * k >= L) rank[k] = 0;
    sum += rank[k];
  }
  if (wave_sum(sum) != L * (L - 1) / 2) {
#pragma unroll
    for (int k = 0; k < K; ++k) tie[lane + kWave * k] = 0;
    KS_LDS_WAIT();  // the counters are clear before any increment
#pragma unroll
    for (int k = 0; k < K; ++k)
      if (lane + kWave * k < L) rank[k] += atomicAdd(&tie[rank[k]], 1);
  }
#pragma unroll
  for (int k = 0; k < K; ++k)
    if (lane + kWave * k < L) gst<T>(out, (uint32_t)(rank[k] * sizeof(T)), v[k]);
}

// One partition of in[s .. s+L-1] into out[s .. s+L-1] by one wave (Steps
// 1-4 on a sub-segment): smaller keys fill upward from s, the others downward
// from s+L-1.  Returns the number of smaller keys.  Four 64-key chunks are
// read before any is written, so one LDS round trip serves four chunks.  The
// valid lanes of a chunk are a prefix of the wave, so a lane's place among
// the other keys is its lane number minus its place among the smaller ones,
// and each lane makes one write.
template <typename T>
__device__ int wave_partition(const T* in, T* out, int s, int L, T key) {
  constexpr int U = 4;
  const int lane = lane_id();
  int cl = 0, cg = 0;
  const int end = s + L;
  for (int base = s + 1; base < end; base += U * kWave) {
    T v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int x = base + u * kWave + lane;
      v[u] = x < end ? in[x] : T(0);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int nv = min(kWave, end - (base + u * kWave));  // valid lanes of this chunk (wave-uniform)
      if (nv > 0) {
        const bool valid = lane < nv;
        const bool lt = valid && !(key <= v[u]);
        const uint64_t bl = __ballot(lt);
        const int r = mbcnt(bl);
        const int d = lt ? s + cl + r : end - 1 - cg - (lane - r);
        if (valid) out[d] = v[u];
        const int nl = __popcll(bl);
        cl += nl;
        cg += nv - nl;
      }
    }
  }
  return cl;
}

// Steps 1-4 on sm.buf[p][s .. s+L-1] by the whole workgroup, into
// sm.buf[p^1][s .. s+L-1]: the keys smaller than the first (the segment's
// key) fill [s, s+c) in position order, the key goes to s+c, where it is
// final (also written to dst), and the others fill (s+c, s+L) in position
// order.  Returns c.  s, L and p are the same in every thread; L <= CUT.
template <typename T, int BLOCK, int CUT>
__device__ int block_partition(FinSmem<T, BLOCK, CUT>& sm, int p, int s, int L, T* dst) {
  constexpr int NW = BLOCK / kWave;
  constexpr int PER = CUT / BLOCK;
  static_assert(CUT % BLOCK == 0 && PER * NW <= kWave, "one wave scans the per-(item, wave) counts");
  const int tid = threadIdx.x, lane = lane_id(), w = tid / kWave;
  const T key = sm.buf[p][s];
  T x[PER];
  uint64_t bl[PER];
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int q = u * BLOCK + tid;
    x[u] = q < L ? sm.buf[p][s + q] : T(0);
  }
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int q = u * BLOCK + tid;
    bl[u] = __ballot(q > 0 && q < L && !(key <= x[u]));
    if (lane == 0) sm.bcnt[u * NW + w] = __popcll(bl[u]);
  }
  __syncthreads();
  if (w == 0) {
    const int c = lane < PER * NW ? sm.bcnt[lane] : 0;
    const int inc = wave_inclusive_scan(c);
    if (lane < PER * NW) sm.bcnt[lane] = inc - c;
    if (lane == kWave - 1) sm.bc = inc;
  }
  __syncthreads();
  const int c = uniform(sm.bc);
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int q = u * BLOCK + tid;
    if (q > 0 && q < L) {
      const int r = sm.bcnt[u * NW + w] + mbcnt(bl[u]);  // smaller keys before q
      const int d = ((bl[u] >> lane) & 1) ? r : c + 1 + (q - 1 - r);
      sm.buf[p ^ 1][s + d] = x[u];
    }
  }
  if (tid == 0) {
    sm.buf[p ^ 1][s + c] = key;
    gst<T>(dst, (uint32_t)((s + c) * sizeof(T)), key);
  }
  __syncthreads();
  return c;
}

__device__ __forceinline__ uint32_t q_entry(int s, int L, int p) {
  return 1u | ((uint32_t)p << 1) | ((uint32_t)s << 2) | ((uint32_t)L << 14);
}

template <typename T, int BLOCK, int CUT>
__device__ void finish_segment(const StageArgs& a, const TaskU& tk, FinSmem<T, BLOCK, CUT>& sm, StageCtr* cur,
                               const Counts& cn, Task* next) {
  constexpr int NW = BLOCK / kWave;
  static_assert(CUT <= 4095, "queue entries hold 12-bit positions and lengths");
  const int tid = threadIdx.x, lane = lane_id();
  const int64_t left = tk.left;
  const int32_t len = (int32_t)tk.len;
  const T* src = (const T*)(tk.parity ? tk.scratch : tk.data) + left;
  T* dst = (T*)tk.data + left;
  const bool want_pivot = tk.root >= 0 && a.pivot_out != nullptr;
  int64_t* pivot_slot = want_pivot ? a.pivot_out + tk.root : nullptr;
  const int64_t pivot_bias = a.pivot_relative ? 0 : left;
  if (len < 1 || len > CUT) {  // never produced by the emitters; guards the LDS arrays
    if (tid == 0) st_agent(&a.flags->overflow, 3);
    if (tid == BLOCK - 1) next->kind = kTaskNone;
    return;
  }

  if (len <= kSmall) {
    // one wave finishes the whole segment in registers
    if (tid < kWave) wave_rank_sort<T>((const KS_GLOBAL T*)src, dst, len, pivot_slot, pivot_bias);
    if (tid == BLOCK - 1) claim_early(a, cur, cn, next);
  } else {
    {
      // all loads in flight before the first LDS store
      constexpr int FI = CUT / BLOCK;
      T v[FI];
#pragma unroll
      for (int k = 0; k < FI; ++k) v[k] = (tid < len - k * BLOCK) ? gld<T>(src + k * BLOCK, (uint32_t)(tid * sizeof(T))) : T(0);
#pragma unroll
      for (int k = 0; k < FI; ++k)
        if (tid < len - k * BLOCK) sm.buf[0][k * BLOCK + tid] = v[k];
    }
    for (int x = tid; x < len + NW + 2; x += BLOCK) sm.q[x] = 0;
    if (tid == 0) {
      sm.q_tail = 0;
      sm.q_head = 0;
      sm.outstanding = 0;
    }
    __syncthreads();
    // The top of the recursion runs on the whole workgroup: the segment
    // itself, then each of its sides of more than kBlockSide keys.  This cuts
    // the chain of large partitions that a single wave would otherwise do
    // alone while the others wait, and the queue starts with up to four
    // sub-segments.  Sides of one key are final.
    auto settle = [&](int s, int L, int p) {  // executed by thread 0
      if (L == 1) {
        gst<T>(dst, (uint32_t)(s * sizeof(T)), sm.buf[p][s]);
      } else if (L >= 2) {
        sm.q[sm.q_tail++] = q_entry(s, L, p);
        ++sm.outstanding;
      }
    };
    const int c1 = block_partition<T, BLOCK, CUT>(sm, 0, 0, len, dst);
    if (tid == 0 && pivot_slot) *pivot_slot = pivot_bias + c1;
#pragma unroll
    for (int side = 0; side < 2; ++side) {
      const int s = side == 0 ? 0 : c1 + 1;
      const int L = side == 0 ? c1 : len - 1 - c1;
      if (L > kBlockSide) {
        const int c2 = block_partition<T, BLOCK, CUT>(sm, 1, s, L, dst);
        if (tid == 0) {
          settle(s, c2, 0);
          settle(s + c2 + 1, L - 1 - c2, 0);
        }
      } else if (tid == 0) {
        settle(s, L, 1);
      }
    }
    __syncthreads();
    // the successor is claimed now, when the queue holds at most four
    // sub-segments for eight waves, so no barrier waits for the claim
    if (tid == BLOCK - 1) claim_early(a, cur, cn, next);
    // Each wave takes sub-segments from the queue until none is outstanding;
    // after a partition it keeps the smaller side for itself and queues the
    // other.  Every branch of this loop is taken on a wave-uniform value
    // (read with readfirstlane before the test): the lanes must stay
    // together for the cross-lane operations inside, and a branch on a
    // per-lane load would let the compiler split them (it may route lanes
    // through different loop exits when it cannot prove a condition uniform).
    uint32_t e = 0;
    for (;;) {
      if (e == 0) {
        int idx = 0;
        if (lane == 0) idx = atomicAdd(&sm.q_head, 1);
        idx = uniform(idx);
        for (;;) {
          e = (uint32_t)uniform((int)__hip_atomic_load(&sm.q[idx], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP));
          if (e != 0) break;
          if (uniform(ld_group(&sm.outstanding)) == 0) break;
          __builtin_amdgcn_s_sleep(1);
        }
        if (e == 0) break;  // everything is done
        KS_MEM_FENCE();  // the side's keys are read only after its entry
      }
      const int p = (e >> 1) & 1, s = (e >> 2) & 0xfff, L = (int)(e >> 14);
      int pushed = 0;
      uint32_t keep = 0;
      if (L <= kLeaf) {
        int32_t* tie = sm.tie[threadIdx.x / kWave];
        if (L <= kWave)
          lds_rank_sort<T, 1>(sm.buf[p] + s, dst + s, L, tie);
        else if (kLeaf <= 2 * kWave || L <= 2 * kWave)
          lds_rank_sort<T, (kLeaf > kWave ? 2 : 1)>(sm.buf[p] + s, dst + s, L, tie);
        else
          lds_rank_sort<T, kLeaf / kWave>(sm.buf[p] + s, dst + s, L, tie);
      } else {
        const T key = sm.buf[p][s];
        const int cl = wave_partition<T>(sm.buf[p], sm.buf[p ^ 1], s, L, key);
        const int cg = L - 1 - cl;
        KS_WAVE_STEP();  // lane 0 and the next partitions read keys the other lanes just wrote
        if (lane == 0) gst<T>(dst, (uint32_t)((s + cl) * sizeof(T)), key);  // Step-4: the key is final
        // Steps 5-6 on the two sides (a side of one key is final)
        if (cl == 1 && lane == 0) gst<T>(dst, (uint32_t)(s * sizeof(T)), sm.buf[p ^ 1][s]);
        if (cg == 1 && lane == 0) gst<T>(dst, (uint32_t)((s + cl + 1) * sizeof(T)), sm.buf[p ^ 1][s + cl + 1]);
        const uint32_t el = cl >= 2 ? q_entry(s, cl, p ^ 1) : 0u;
        const uint32_t eg = cg >= 2 ? q_entry(s + cl + 1, cg, p ^ 1) : 0u;
        pushed = (el != 0) + (eg != 0);
        // keep the smaller side, queue the other
        const bool keep_lt = el != 0 && (eg == 0 || cl <= cg);
        keep = keep_lt ? el : eg;
        const uint32_t give = keep_lt ? eg : el;
        if (give != 0) {
          // the side's keys (written by this wave) are in LDS before its entry
          KS_LDS_WAIT();
          if (lane == 0) {
            const int qi = atomicAdd(&sm.q_tail, 1);
            __hip_atomic_store(&sm.q[qi], give, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
          }
        }
      }
      // new entries are written before this update
      KS_LDS_WAIT();
      if (lane == 0)
        __hip_atomic_fetch_add(&sm.outstanding, pushed - 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      e = (uint32_t)uniform((int)keep);
    }
    __syncthreads();
  }
  if (tid == 0 && a.pending) {
    const int32_t old = add_agent(a.pending + tk.buf, -1);
    if (old - 1 == 0 && a.done_stage) st_agent(a.done_stage + tk.buf, a.stage);
  }
  if (tid == BLOCK - 1 && next->kind == kTaskUnclaimed) fetch_task(a, cur, cn, next);
}

// ---------------------------------------------------------------------------
// the stage kernel: a persistent grid drains the stage's tickets

template <typename T, int BLOCK, int ITEMS, int CUT>
__global__ __launch_bounds__(BLOCK) void stage_kernel(StageArgs a) {
  __shared__ StageSmem<T, BLOCK, ITEMS, CUT> sm;
  __shared__ Task next;
  __shared__ int32_t s_counts[4];
  StageCtr* cur = a.ctr + (a.stage % 3);
  StageCtr* nx = a.ctr + ((a.stage + 1) % 3);
  if (threadIdx.x == BLOCK - 1) {
    if (blockIdx.x == 0) {
      StageCtr* nn = a.ctr + ((a.stage + 2) % 3);
      st_agent(&nn->nseg, 0);
      st_agent(&nn->ntiles, 0);
      st_agent(&nn->nfin, 0);
      st_agent(&nn->ticket, 0);
      st_agent(&nn->carry, 0);
    }
    // after a failed consistency check the lists may be incomplete: do
    // nothing (the host reports the error)
    const int32_t ovf = ld_agent(&a.flags->overflow);
    const int32_t nt = min(ld_agent(&cur->ntiles), a.cap_tiles);
    const int32_t ncar = min(ld_agent(&cur->carry), a.cap_fin - a.fin_half);
    const int32_t nf = ncar + min(ld_agent(&cur->nfin), a.fin_half);
    // A stage that also partitions runs at most fin_run finish tasks, one
    // round on the grid; the rest wait for the next stage, whose partitions
    // are fewer, instead of a second round that would end this stage late.
    const int32_t ndef = nt > 0 && nf > a.fin_run ? min(nf - a.fin_run, a.cap_fin - a.fin_half) : 0;
    const Counts cn{nt, nt + nf - ndef, ncar};
    next.bnext = next.bend = 0;
    if (ovf != 0)
      next.kind = kTaskNone;
    else
      fetch_task(a, cur, cn, &next, a.fixed_first ? (int32_t)blockIdx.x : -1);
    s_counts[0] = cn.ntiles;
    s_counts[1] = cn.nwork;
    s_counts[2] = cn.ncar;
    s_counts[3] = ovf != 0 ? 0 : ndef;
  }
  __syncthreads();
  const Counts cn{uniform(s_counts[0]), uniform(s_counts[1]), uniform(s_counts[2])};
  const int32_t ndef = uniform(s_counts[3]);
  if (ndef > 0) {
    // carry the deferred finish tasks (the last ndef finish tickets) into
    // the upper half of the next stage's finish list
    const int par = a.stage & 1;
    const int32_t nrun = cn.nwork - cn.ntiles;
    int64_t carried = 0;  // keys of the tasks this thread carried
    for (int32_t j = blockIdx.x * BLOCK + threadIdx.x; j < ndef; j += gridDim.x * BLOCK) {
      Seg d;
      load_seg(&d, (const KS_GLOBAL Seg*)a.fin[par] + fin_slot(a, cn, nrun + j));
      store_seg((KS_GLOBAL Seg*)a.fin[par ^ 1] + a.fin_half + j, d);
      carried += d.len;
    }
    if (a.stage_keys && a.stage + 1 < a.cap_stats) {
      // profiling: the carried keys move from this stage's count to the
      // next one's, with one pair of global atomics per workgroup (two per
      // task cost as much as a pass when a quarter of a million wait)
      __shared__ unsigned long long s_carried;
      if (threadIdx.x == 0) s_carried = 0;
      __syncthreads();
      if (carried) atomicAdd(&s_carried, (unsigned long long)carried);
      __syncthreads();
      if (threadIdx.x == 0 && s_carried) {
        atomicAdd((unsigned long long*)&a.stage_keys[2 * (a.stage + 1) + 1], s_carried);
        atomicAdd((unsigned long long*)&a.stage_keys[2 * a.stage + 1], (unsigned long long)(-(int64_t)s_carried));
      }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      st_agent(&nx->carry, ndef);
      atomicMax(&a.flags->last_active, a.stage + 1);
    }
  }
  for (;;) {
    const TaskU tk = read_task(&next);
    __syncthreads();  // everyone has read `next` before it is overwritten
    if (tk.kind == kTaskNone) break;
    if (tk.kind == kTaskTile)
      partition_tile<T, BLOCK, ITEMS>(a, tk, sm.p, cur, cn, &next);
    else
      finish_segment<T, BLOCK, CUT>(a, tk, sm.f, cur, cn, &next);
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// set-up kernels

// Zero-fills n 64-bit words (look-back words before a run).
__global__ void clear_kernel(uint64_t* p, int64_t n) {
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x)
    p[j] = 0;
}

// Clears the look-back words, counters and flags before a run (one kernel:
// each boundary between kernels costs a few microseconds).
__global__ void reset_kernel(StageCtr* ctr, Flags* flags, uint64_t* status, int64_t nwords) {
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < nwords; j += (int64_t)gridDim.x * blockDim.x)
    status[j] = 0;
  if (blockIdx.x != 0) return;
  const int tid = threadIdx.x;
  if (tid < 3) {
    ctr[tid].nseg = 0;
    ctr[tid].ntiles = 0;
    ctr[tid].nfin = 0;
    ctr[tid].ticket = 0;
    ctr[tid].carry = 0;
  }
  if (tid == 0) {
    flags->last_active = -1;
    flags->err = 0;
    flags->overflow = 0;
    flags->diag_stage = -1;
    flags->diag_tile = -1;
    flags->diag_pred = -1;
    flags->diag_word = 0;
  }
}

// One block per input array (or per segment in single-level mode): validate,
// classify into the lists of stage a.stage (0 for a fresh run; the server
// admits requests into its current stage) and write the tile map.
__global__ void init_kernel(InitArgs ia) {
  __shared__ int32_t s_slot, s_first, s_nt;
  const StageArgs& a = ia.sa;
  const int64_t u = blockIdx.x;
  const int tid = threadIdx.x;
  int64_t left, len;
  if (ia.offsets) {
    left = ia.offsets[u];
    len = ia.offsets[u + 1] - left;
  } else if (ia.seg_left) {
    left = ia.seg_left[u];
    len = ia.seg_len[u];
  } else {
    left = 0;
    len = ia.n;
  }
  const bool bad = left < 0 || len < 0 || left > ia.n || len > ia.n - left || (ia.level_mode && len < 1);
  if (bad) {
    if (tid == 0) st_agent(&a.flags->err, 1);
    return;
  }
  const int par = a.stage & 1;
  StageCtr* c0 = a.ctr + (a.stage % 3);
  const int32_t root = ia.root_base + (int32_t)u;
  if (tid == 0) {
    s_nt = 0;
    int nseg = 0;
    if (a.pending && u == 0) {
      st_agent(a.pending + ia.buf, 0);
      if (a.done_stage) st_agent(a.done_stage + ia.buf, -1);
    }
    Seg d;
    d.left = left;
    d.len = len;
    d.data = ia.pair.data;
    d.scratch = ia.pair.scratch;
    d.root = root;
    d.buf = ia.buf;
    d.parity = ia.level_mode ? 1 : 0;
    d.first_tile = 0;
    if (len == 0) {
      if (a.pivot_out) a.pivot_out[root] = -1;
    } else if (!ia.level_mode && len <= a.cutoff) {
      const int32_t f = add_agent(&c0->nfin, 1);
      if (f < a.fin_half) {
        a.fin[par][f] = d;
        ++nseg;
        if (a.stage_keys && a.stage < a.cap_stats)
          atomicAdd((unsigned long long*)&a.stage_keys[2 * a.stage + 1], (unsigned long long)len);
      } else {
        st_agent(&a.flags->overflow, 1);
      }
    } else {
      const int32_t nt = (int32_t)((len + ia.tile - 1) / ia.tile);
      const int32_t s = add_agent(&c0->nseg, 1);
      const int32_t f = add_agent(&c0->ntiles, nt);
      if (s < a.cap_live && f + nt <= a.cap_tiles) {
        d.first_tile = f;
        a.live[par][s] = d;
        s_slot = s;
        s_first = f;
        s_nt = nt;
        ++nseg;
        if (a.stage_keys && a.stage < a.cap_stats)
          atomicAdd((unsigned long long*)&a.stage_keys[2 * a.stage], (unsigned long long)len);
      } else {
        st_agent(&a.flags->overflow, 1);
      }
    }
    if (nseg) atomicMax(&a.flags->last_active, a.stage);
    if (a.pending && nseg) add_agent(a.pending + ia.buf, nseg);
  }
  __syncthreads();
  const int32_t nt = s_nt;
  if (nt > 0) {
    int32_t* tm = a.tilemap[par] + s_first;
    const int32_t s = s_slot;
    for (int j = tid; j < nt; j += blockDim.x) tm[j] = s;
  }
}

}  // namespace ksort
