// The literal arrangement of Steps 1-4 (arXiv 1107.3622, Section 1.1) on
// the GPU, one level at a time.
//
// The fast path places the keys of each side in an order of its own; here
// every level leaves exactly the array the sequential steps leave, so every
// later key, call and pivot index is the paper's.  The arrangement of one
// call on [left, right] with key = a[left] has a closed form:
//   c = #{x in (left, right] : a[x] < key} and i = left + c (Step-4);
//   m = i + 1 if i < right and a[i+1] >= key, else m = i;
//   q_1 < q_2 < ... are the positions in (left, m] holding a key >= key and
//   r_1 > r_2 > ... the positions in (m, right] holding a key < key (there
//   are as many as q's, or one fewer);
//   the key goes to i and a[q_1] (the Step-3.1 temp) to i + 1; a smaller key
//   at x <= m moves to x - 1; a larger-or-equal key at x > m stays; a[q_k]
//   goes to r_{k-1} (k >= 2) and a[r_k] to q_k - 1.
// (Step-3.2 shifts the smaller keys met before the scan and the descending
// pointer cross down by one; Step-3.1 swaps each larger key it meets there
// with the smaller key the descending pointer found, Hoare-style.)
//
// Everything follows from one number per position: the count of smaller
// keys from its segment's start up to it (a segmented scan).  A level is
//   scan_level  : that count, in ltp[] (one pass, decoupled look-back), and
//                 in a whole sort the list of blocks not idle this level;
//   move_kernel : keys that shift or stay, and the q and r keys filed by rank;
//   pair_kernel : q_k -> r_{k-1} and r_k -> q_k - 1, the call record, and the
//                 segments of the next level (Steps 5-6);
//   small_kernel: in a whole sort, every remaining call on the sides of at
//                 most 64 keys, one wave per side.
// Per position the state is hd[x], the first position of its segment (-1 if
// the key is final or outside every segment), and, at a segment's first
// position, ln[x], its length.  Positions are 32-bit: n < 2^31.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <memory>
#include <mutex>
#include <vector>

#include "ksort_engine.h"

namespace ksort {
namespace exact {

// Waits for this wave's LDS accesses: lanes of a wave read what other lanes
// of it wrote just before (a wave executes in step).
#ifndef KS_LDS_WAIT
#define KS_LDS_WAIT() asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory")
#endif

constexpr int kThreads = 256;
constexpr int kItems = 16;
constexpr int kSpan = kThreads * kItems;  // positions per scan block
constexpr int kShort = 64;                // sort mode: sides of at most this many keys finish in one wave
constexpr int kPairGrid = 4096;           // most workgroups of move_kernel and pair_kernel
// Workgroups of small_kernel (7e6 keys: 512, 1024, 2048, 4096 and 8192 took
// 6.18, 5.90, 5.78, 5.81 and 5.83 ms per sort).
constexpr int kSmallGrid = 2048;

template <typename T>
struct LevelArgs {
  const T* cur;            // keys before this level
  T* nxt;                  // keys after it
  const int32_t* hd;       // segment start of each position, or -1
  const int32_t* ln;       // length, at segment starts
  int32_t* hd2;            // next level (sort mode only)
  int32_t* ln2;
  int32_t* ltp;            // smaller keys from the segment start through the position
  int32_t* qpos;           // position of q_k, at segment start + k
  int32_t* rpos;           // position of r_k, at segment start + k
  T* qkey;
  T* rkey;
  uint64_t* sstat[2];      // per scan block, by level parity: its published run (look-back word)
  int32_t* sctr;           // two ticket counters, by level parity
  int32_t* err;            // set when a look-back wait gives up
  int32_t par;             // this level's parity
  uint32_t spin_limit;     // polls of a look-back wait before it gives up
  int64_t n;
  int32_t nblocks;
  int32_t sort_mode;       // 1: whole-array sort (final keys copied, next level built)
  int32_t* piv_at;         // level mode: i of the segment starting at each position
  int64_t* calls;          // (left, right, i) per call, in no particular order
  int64_t calls_cap;
  unsigned long long* ncalls;
  // sort mode without call records: per-workgroup call counts, one slot per
  // workgroup of pair_kernel (kPairSlots) and of small_kernel after them;
  // each slot belongs to one workgroup index, so plain adds suffice
  unsigned long long* wcalls;
  int64_t* first_pivot;    // set by the call on [0, n-1] when not null
  unsigned long long* active;  // positions in segments of two or more keys next level
  // sort mode: per scan block, whether any of its positions is in a segment
  // at this level, at the level before, and (written here) at the next one;
  // null in level mode (nothing is skipped)
  const uint8_t* act;
  const uint8_t* act_prev;
  uint8_t* act_next;
  // sort mode: the blocks that are not idle this level (see block_idle),
  // listed by scan_level in claim order, and their number, by level parity;
  // move_kernel and pair_kernel walk quarter blocks of this list only.
  // Each count has a cache line of its own: one is cleared with a plain
  // store while the other takes atomic adds.  Null in level mode.
  int32_t* blist[2];
  int32_t* nblist[2];
  // sort mode: sides of 2 .. kShort keys filed this level as (left, len),
  // in ngroups lists of small_cap entries each, one per group of
  // consecutive pair_kernel workgroups (npair of them), with the lengths in
  // nsmall[group]; small_kernel makes all their remaining calls.  Null in
  // level mode.
  int2* small;
  int32_t* nsmall;
  int64_t small_cap;
  int32_t npair;
  int32_t ngroups;
};

// Lists of short sides: one shared counter for all pair_kernel workgroups
// serializes their additions (a device-scope atomic on one address serves
// a few tens of millions per second); one list per workgroup leaves
// small_kernel unbalanced.  kSmallGroups lists, each shared by a group of
// consecutive workgroups, keep both small.
constexpr int kSmallGroups = 256;

// A block whose positions are all final at this level and the one before
// holds the same keys and segment state in both buffers: nothing to do.
template <typename T>
__device__ __forceinline__ bool block_idle(const LevelArgs<T>& a, int64_t b) {
  return a.act && !a.act[b] && !a.act_prev[b];
}

// Reads the block list or its count, written by the kernel before, with
// an agent-scope load, as the list was written (the address is the same in
// every lane, and a plain load of it may be made a scalar load).
__device__ __forceinline__ int32_t list_load(const int32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Work unit of move_kernel and pair_kernel in sort mode: a quarter of a
// listed block, kUnit / kThreads rounds of the workgroup.  Idle blocks are
// not listed, so nearly idle levels cost little more than their launches.
constexpr int kUnit = kSpan / 4;
static_assert(kUnit % kThreads == 0, "whole rounds per unit");

// (flag, sum) pairs: a flag starts a new run; sum counts smaller keys.
struct Run {
  int f, s;
};
__device__ __forceinline__ Run join(Run a, Run b) { return Run{a.f | b.f, b.f ? b.s : a.s + b.s}; }

// The pair of position x: a segment start (or a final key) begins a run and
// counts nothing; any other position counts 1 if its key is smaller than
// its segment's key.  Comparisons are exactly `key <= a[x]` (ties go right).
template <typename T>
__device__ __forceinline__ Run pos_run(const LevelArgs<T>& a, int64_t x) {
  if (x >= a.n) return Run{1, 0};
  const int32_t h = a.hd[x];
  if (h < 0 || h == x) return Run{1, 0};
  return Run{0, !(a.cur[h] <= a.cur[x]) ? 1 : 0};
}

// Look-back word of a scan block: the smaller-key count in bits 0..31, the
// run flag (a segment starts in the block) in bit 32, and in bits 33..34
// what the word holds: 1 the block's own run, 2 the run from the array's
// start through the block.  0 means not yet published; each level clears the
// words of the level after it.
constexpr uint64_t kRunOwn = 1, kRunIncl = 2;
__device__ __forceinline__ uint64_t run_word(uint64_t kind, Run r) {
  return (kind << 33) | ((uint64_t)(r.f & 1) << 32) | (uint32_t)r.s;
}
__device__ __forceinline__ Run word_run(uint64_t w) { return Run{(int)((w >> 32) & 1), (int)(uint32_t)w}; }

// Scan blocks a workgroup takes with one ticket.  One ticket per block cost
// about 15 ns of serialized device-scope atomics each (24 us per level at
// 7e6 keys, also in levels that are nearly idle).
constexpr int kScanChunk = 4;

// Inclusive scan of K Run pairs per thread across the workgroup, each of
// the K sequences on its own: within each wave by shuffles, then each wave
// joins the totals of the waves before it (one barrier).  The results are
// also left in sf/ss (by sequence and thread) for the caller.
template <int K>
__device__ void block_scan_k(Run (&r)[K], int (*sf)[kThreads], int (*ss)[kThreads]) {
  constexpr int NW = kThreads / 64;
  __shared__ int wf[K][NW], wsum[K][NW];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    for (int d = 1; d < 64; d <<= 1) {
      const int pf = __shfl_up(r[k].f, d), ps = __shfl_up(r[k].s, d);
      if (lane >= d) r[k] = join(Run{pf, ps}, r[k]);
    }
    if (lane == 63) {
      wf[k][w] = r[k].f;
      wsum[k][w] = r[k].s;
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < K; ++k) {
    Run pre{0, 0};  // the identity of join
    for (int j = 0; j < w; ++j) pre = join(pre, Run{wf[k][j], wsum[k][j]});
    r[k] = join(pre, r[k]);
    sf[k][t] = r[k].f;
    ss[k][t] = r[k].s;
  }
  __syncthreads();
}

// The count of smaller keys from each position's segment start through it,
// in one pass.  Each workgroup takes the next kScanChunk scan blocks in
// claim order, so every block it waits for belongs to a workgroup that has
// started.  It scans the kItems x kThreads positions of each, publishes every
// block's own run at once, finds the run carried into its first block by
// decoupled look-back (the nearest earlier block that has published its run
// from the array's start, or that contains a segment start, ends it), and
// from that the runs from the array's start through each of its blocks.
// The first workgroup of a level also clears the level's counters (active
// positions, filed sides) and the next level's ticket counter.
template <typename T>
__global__ __launch_bounds__(kThreads) void scan_level(LevelArgs<T> a) {
  constexpr int K = kScanChunk;
  __shared__ int sf[K][kThreads], ss[K][kThreads];
  __shared__ int s_b, s_pf[K], s_ps[K];
  if (threadIdx.x == 0) {
    const int c = atomicAdd(a.sctr + a.par, 1);
    s_b = c * K;
    if (c == 0) {
      a.sctr[a.par ^ 1] = 0;
      if (a.active) *a.active = 0;
      if (a.nblist[0]) *a.nblist[a.par ^ 1] = 0;  // the next level's list
      if (a.nsmall)
        for (int g = 0; g < a.ngroups; ++g) a.nsmall[g] = 0;  // (one thread: at most kSmallGroups stores)
    }
    if (a.nblist[0]) {
      // list the chunk's blocks that are not idle (one atomic per chunk;
      // a bit mask, not an array indexed by a running count, which the
      // device compiler was seen to fill wrongly here)
      uint32_t m = 0;
#pragma unroll
      for (int k = 0; k < K; ++k)
        if (c * K + k < a.nblocks && !block_idle(a, c * K + k)) m |= 1u << k;
      if (m) {
        int32_t at = atomicAdd(a.nblist[a.par], __builtin_popcount(m));
        for (int k = 0; k < K; ++k)
          if ((m >> k) & 1) __hip_atomic_store(a.blist[a.par] + at++, (int32_t)(c * K + k), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
  }
  __syncthreads();
  const int64_t b0 = s_b;
  uint64_t* st = a.sstat[a.par];
  bool live[K];      // the block exists and has a position in a segment
  uint32_t fbits[K], lbits[K];  // per item: run start, smaller key
  Run r[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int64_t blk = b0 + k;
    live[k] = blk < a.nblocks && (!a.act || a.act[blk]);
    fbits[k] = lbits[k] = 0;
    r[k] = Run{1, 0};  // a block that is missing or all final: a run start counting nothing
    if (blk < a.nblocks && threadIdx.x == 0) {
      a.sstat[a.par ^ 1][blk] = 0;  // the next level's word starts unpublished
      if (a.act) a.act_next[blk] = 0;
    }
  }
  bool any_live = false;
#pragma unroll
  for (int k = 0; k < K; ++k) any_live = any_live || live[k];
  if (!any_live) {
    // every block of the chunk is a run start counting nothing whatever
    // comes before it: its run from the array's start is its own, published
    // at once; nothing reads its counts
    if (threadIdx.x == 0)
#pragma unroll
      for (int k = 0; k < K; ++k)
        if (b0 + k < a.nblocks)
          __hip_atomic_store(st + b0 + k, run_word(kRunIncl, Run{1, 0}), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return;
  }
  // The positions are read striped (item j of every thread at j * kThreads
  // + t, so each load of a wave covers consecutive positions), and each
  // position's two bits reach the thread that scans it (kItems consecutive
  // positions from t * kItems) through the waves' ballots, kept in LDS.
  static_assert(kItems == 16 && kThreads == 256, "the bit exchange below assumes 16 rows of 256 positions");
  __shared__ uint64_t s_fm[K][kItems][kThreads / 64], s_lm[K][kItems][kThreads / 64];
  {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      if (!live[k]) continue;
      const int64_t base = (b0 + k) * kSpan + threadIdx.x;
      if ((b0 + k + 1) * kSpan <= a.n) {
        int32_t h[kItems];
        T v[kItems];
#pragma unroll
        for (int j = 0; j < kItems; ++j) {
          h[j] = a.hd[base + j * kThreads];
          v[j] = a.cur[base + j * kThreads];
        }
#pragma unroll
        for (int j = 0; j < kItems; ++j) {
          const bool start = h[j] < 0 || h[j] == base + j * kThreads;
          const bool lt = !start && !(a.cur[h[j]] <= v[j]);
          const uint64_t fm = __ballot(start), lm = __ballot(lt);
          if (lane == 0) {
            s_fm[k][j][wv] = fm;
            s_lm[k][j][wv] = lm;
          }
        }
      } else {
#pragma unroll
        for (int j = 0; j < kItems; ++j) {
          const Run p = pos_run(a, base + j * kThreads);
          const uint64_t fm = __ballot(p.f != 0), lm = __ballot(p.s != 0);
          if (lane == 0) {
            s_fm[k][j][wv] = fm;
            s_lm[k][j][wv] = lm;
          }
        }
      }
    }
  }
  __syncthreads();
  {
    // thread t's positions t * 16 .. t * 16 + 15: row t / 16, wave
    // (t % 16) / 4 of that row, bits (t % 4) * 16 ..
    const int t = threadIdx.x, row = t >> 4, w = (t & 15) >> 2, sh = (t & 3) * 16;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      if (!live[k]) continue;
      fbits[k] = (uint32_t)(s_fm[k][row][w] >> sh) & 0xffffu;
      lbits[k] = (uint32_t)(s_lm[k][row][w] >> sh) & 0xffffu;
      r[k] = Run{0, 0};
#pragma unroll
      for (int j = 0; j < kItems; ++j) r[k] = join(r[k], Run{(int)((fbits[k] >> j) & 1), (int)((lbits[k] >> j) & 1)});
    }
  }
  block_scan_k<K>(r, sf, ss);
  if (threadIdx.x < 64) {
    const int lane = threadIdx.x;
    // every block's own run first, so later workgroups can look back
    // across this chunk while its first block waits
    if (lane < K && b0 + lane < a.nblocks && b0 + lane > 0) {
      const Run agg{sf[lane][kThreads - 1], ss[lane][kThreads - 1]};
      __hip_atomic_store(st + b0 + lane, run_word(kRunOwn, agg), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    Run pre{0, 0};
    if (b0 > 0) {
      int64_t top = b0 - 1;  // lane j watches block top - j
      int sum = 0;
      uint32_t polls = 0;
      for (;;) {
        const int64_t j = top - lane;
        uint64_t w = j >= 0 ? __hip_atomic_load(st + j, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0;
        // wait until every watched block has published
        while (__ballot(j >= 0 && (w >> 33) == 0)) {
          if (++polls > a.spin_limit) break;
          __builtin_amdgcn_s_sleep(1);
          if (j >= 0 && (w >> 33) == 0) w = __hip_atomic_load(st + j, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        if (polls > a.spin_limit) {
          if (lane == 0) atomicExch(a.err, 1);
          pre = Run{1, 0};
          break;
        }
        // the nearest block whose word ends the look-back: a run from the
        // array's start, or a run with a segment start in it
        const bool stop = j >= 0 && ((w >> 33) == kRunIncl || ((w >> 32) & 1));
        const uint64_t sm = __ballot(stop);
        const int first_stop = sm ? __builtin_ctzll(sm) : 64;
        const Run wr = word_run(w);
        int part = j >= 0 && lane < first_stop ? wr.s : 0;
        for (int d = 32; d > 0; d >>= 1) part += __shfl_xor(part, d);
        sum += part;
        if (sm) {
          const uint64_t ws = __shfl(w, first_stop);
          const Run rs = word_run(ws);
          pre = Run{rs.f, rs.s + sum};
          break;
        }
        top -= 64;
      }
    }
    // runs from the array's start through each block of the chunk
    if (lane == 0) {
      Run acc = pre;
#pragma unroll
      for (int k = 0; k < K; ++k) {
        s_pf[k] = acc.f;
        s_ps[k] = acc.s;
        acc = join(acc, Run{sf[k][kThreads - 1], ss[k][kThreads - 1]});
        if (b0 + k < a.nblocks)
          __hip_atomic_store(st + b0 + k, run_word(kRunIncl, acc), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < K; ++k) {
    if (!live[k]) continue;
    const int64_t base = (b0 + k) * kSpan + (int64_t)threadIdx.x * kItems;
    Run run = join(Run{s_pf[k], s_ps[k]}, threadIdx.x > 0 ? Run{sf[k][threadIdx.x - 1], ss[k][threadIdx.x - 1]} : Run{0, 0});
    int32_t out[kItems];
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
      run = join(run, Run{(int)((fbits[k] >> j) & 1), (int)((lbits[k] >> j) & 1)});
      out[j] = run.s;
    }
    if (base + kItems <= a.n) {
#pragma unroll
      for (int q = 0; q < kItems / 4; ++q)
        *(int4*)(a.ltp + base + 4 * q) = make_int4(out[4 * q], out[4 * q + 1], out[4 * q + 2], out[4 * q + 3]);
    } else {
#pragma unroll
      for (int j = 0; j < kItems; ++j)
        if (base + j < a.n) a.ltp[base + j] = out[j];
    }
  }
}

// The quantities of the call on the segment starting at h.
template <typename T>
struct Call {
  int64_t left, right, c, i, m;
  T key;
};
template <typename T>
__device__ __forceinline__ Call<T> call_of(const LevelArgs<T>& a, int32_t h) {
  Call<T> k;
  k.left = h;
  k.right = h + (int64_t)a.ln[h] - 1;
  k.key = a.cur[h];
  k.c = a.ltp[k.right];
  k.i = k.left + k.c;
  k.m = (k.i < k.right && k.key <= a.cur[k.i + 1]) ? k.i + 1 : k.i;
  return k;
}

// call_of for any position of a listed block: a final position (h < 0)
// gets a call on itself, with every index kept inside the array, whose
// numbers are never used.  So the loads of several rounds can all be
// issued before any branch on them.  For h >= 0 it equals call_of.
__device__ __forceinline__ int64_t clamp64(int64_t v, int64_t lo, int64_t hi) { return v < lo ? lo : v > hi ? hi : v; }
template <typename T>
__device__ __forceinline__ Call<T> call_any(const LevelArgs<T>& a, int32_t h, int64_t x) {
  Call<T> k;
  const int64_t last = a.n - 1;
  k.left = h < 0 ? x : h;
  k.right = clamp64(k.left + (int64_t)a.ln[k.left] - 1, k.left, last);
  k.key = a.cur[k.left];
  k.c = a.ltp[k.right];
  k.i = clamp64(k.left + k.c, k.left, k.right);
  const T after = a.cur[k.i < last ? k.i + 1 : last];
  k.m = (k.i < k.right && k.key <= after) ? k.i + 1 : k.i;
  return k;
}

// The moves of position x in segment h (h >= 0) with call k: v = cur[x],
// lp = ltp[x].  For a final position (h < 0, sort mode) lp is hd2[x]: the
// key is copied if it was in a segment the level before.
template <typename T>
__device__ __forceinline__ void move_apply(const LevelArgs<T>& a, int64_t x, int32_t h, const Call<T>& k, T v,
                                           int32_t lp) {
  if (h < 0) {
    if (lp >= 0) a.nxt[x] = v;
    return;
  }
  if (x == k.left) {
    a.nxt[k.i] = k.key;
    return;
  }
  const bool lt = !(k.key <= v);
  if (x <= k.m) {
    if (lt) {
      a.nxt[x - 1] = v;
    } else {
      const int64_t r = (x - k.left) - lp;  // rank among the keys >= key in (left, x]
      if (r == 1)
        a.nxt[k.i + 1] = v;
      else
        a.qkey[k.left + r] = v;
      a.qpos[k.left + r] = (int32_t)x;
    }
  } else {
    if (!lt) {
      a.nxt[x] = v;
    } else {
      const int64_t r = k.c - lp + 1;  // rank among the smaller keys in [x, right]
      a.rpos[k.left + r] = (int32_t)x;
      a.rkey[k.left + r] = v;
    }
  }
}

template <typename T>
__device__ __forceinline__ void move_one(const LevelArgs<T>& a, int64_t x) {
  const int32_t h = a.hd[x];
  if (h < 0) {
    // a key that became final in the level before is copied once; both
    // buffers hold it from then on (hd2 still holds that level's state)
    if (a.sort_mode && (!a.act || a.hd2[x] >= 0)) a.nxt[x] = a.cur[x];
    return;
  }
  move_apply(a, x, h, call_of(a, h), a.cur[x], a.ltp[x]);
}

template <typename T>
__global__ __launch_bounds__(kThreads) void move_kernel(LevelArgs<T> a) {
  if (a.nblist[0]) {
    const int64_t nu = 4 * (int64_t)list_load(a.nblist[a.par]);
    const int32_t* bl = a.blist[a.par];
    for (int64_t u = blockIdx.x; u < nu; u += gridDim.x) {
      const int64_t base = (int64_t)list_load(bl + (u >> 2)) * kSpan + (u & 3) * kUnit;
      // the unit's rounds load everything first (their chains of dependent
      // loads overlap), then store
      constexpr int R = kUnit / kThreads;
      int64_t xs[R];
      int32_t hs[R], lps[R];
      T vs[R];
      Call<T> ks[R];
#pragma unroll
      for (int j = 0; j < R; ++j) {
        xs[j] = base + j * kThreads + threadIdx.x;
        hs[j] = a.hd[xs[j] < a.n ? xs[j] : a.n - 1];
      }
#pragma unroll
      for (int j = 0; j < R; ++j) {
        const int64_t xc = xs[j] < a.n ? xs[j] : a.n - 1;
        ks[j] = call_any(a, hs[j], xc);
        vs[j] = a.cur[xc];
        lps[j] = (hs[j] < 0 ? a.hd2 : a.ltp)[xc];  // (sort mode: hd2 is there)
      }
#pragma unroll
      for (int j = 0; j < R; ++j)
        if (xs[j] < a.n) move_apply(a, xs[j], hs[j], ks[j], vs[j], lps[j]);
    }
    return;
  }
  for (int64_t x = (int64_t)blockIdx.x * kThreads + threadIdx.x; x < a.n; x += (int64_t)gridDim.x * kThreads)
    if (!block_idle(a, x / kSpan)) move_one(a, x);
}

template <typename T>
__global__ __launch_bounds__(kThreads) void pair_kernel(LevelArgs<T> a) {
  unsigned long long ncall = 0;
  bool any_active = false;
  const int lane = threadIdx.x & 63;
  // this workgroup's list of short sides (sort mode)
  const int32_t grp = a.small ? (int32_t)((int64_t)blockIdx.x * a.ngroups / a.npair) : 0;
  // One round: the kThreads positions from base.  Every thread of a
  // workgroup runs the same rounds (the bounds are on the round's first
  // position) and the waves file their short sides on their own, so nothing
  // in a round waits for the other waves.
  // h, k and lm (= ltp[k.m]) are the round's position's loads (call_any).
  auto round = [&](int64_t base, int32_t h, const Call<T>& k, int32_t lm) {
    const int64_t x = base + threadIdx.x;
    bool file = false;
    int2 entry{0, 0};
    if (x < a.n) {
      if (h < 0) {
        if (a.sort_mode) a.hd2[x] = -1;
      } else {
        const int64_t nq = (k.m - k.left) - lm;  // keys >= key in (left, m]
        const int64_t nr = k.c - lm;             // smaller keys in (m, right]
        const int64_t r = x - k.left;
        // (the slots read here were filed by move_kernel in this level: the
        // closed form has nr = nq or nq - 1; the range checks only keep a
        // corrupted slot from writing outside the segment)
        if (r >= 2 && r <= nq) {
          const int64_t to = a.rpos[k.left + r - 1];
          if (to > k.left && to <= k.right) a.nxt[to] = a.qkey[k.left + r];
        }
        if (r >= 1 && r <= nr) {
          const int64_t to = (int64_t)a.qpos[k.left + r] - 1;
          if (to >= k.left && to <= k.right) a.nxt[to] = a.rkey[k.left + r];
        }
        if (r == 0) {
          // a call: with records wanted, each takes a slot (and so is
          // counted); otherwise it is counted in the workgroup's slot
          if (a.calls) {
            const unsigned long long j = atomicAdd(a.ncalls, 1ull);
            if ((int64_t)j < a.calls_cap) {
              a.calls[3 * j] = k.left;
              a.calls[3 * j + 1] = k.right;
              a.calls[3 * j + 2] = k.i;
            }
          } else {
            ++ncall;
          }
          if (a.piv_at) a.piv_at[k.left] = (int32_t)k.i;
          if (a.first_pivot && k.left == 0 && k.right == a.n - 1) *a.first_pivot = k.i;
        }
        if (a.sort_mode) {
          // Steps 5-6: [left, i-1] and [i+1, right] go on if they hold two
          // or more keys; a side of at most kShort keys is filed for
          // small_kernel (its first position files it) and its positions
          // leave the levels
          int32_t nh = -1;
          const int64_t cr = k.right - k.i;
          if (x < k.i && k.c >= 2) {
            if (a.small && k.c <= kShort) {
              file = x == k.left;
              entry = make_int2((int32_t)k.left, (int32_t)k.c);
            } else {
              nh = (int32_t)k.left;
            }
          }
          if (x > k.i && cr >= 2) {
            if (a.small && cr <= kShort) {
              file = x == k.i + 1;
              entry = make_int2((int32_t)(k.i + 1), (int32_t)cr);
            } else {
              nh = (int32_t)(k.i + 1);
            }
          }
          a.hd2[x] = nh;
          if (nh == x) a.ln2[x] = (int32_t)(x == k.left ? k.c : k.right - k.i);
          if (nh >= 0) {
            any_active = true;
            if (a.act_next) a.act_next[x / kSpan] = 1;
          }
        }
      }
    }
    if (a.small) {
      // the wave's filed sides take one range of its group's list (one
      // atomic per wave with sides to file; no workgroup barrier)
      const uint64_t fm = __ballot(file);
      if (fm) {
        int32_t at = 0;
        if (lane == 0) at = atomicAdd(a.nsmall + grp, (int32_t)__popcll(fm));
        at = __shfl(at, 0);
        if (file)
          a.small[grp * a.small_cap + at +
                  __builtin_amdgcn_mbcnt_hi((uint32_t)(fm >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)fm, 0))] = entry;
      }
    }
  };
  if (a.nblist[0]) {
    const int64_t nu = 4 * (int64_t)list_load(a.nblist[a.par]);
    const int32_t* bl = a.blist[a.par];
    for (int64_t u = blockIdx.x; u < nu; u += gridDim.x) {
      const int64_t b0 = (int64_t)list_load(bl + (u >> 2)) * kSpan + (u & 3) * kUnit;
      // every round's chain of loads first, so that they overlap
      constexpr int R = kUnit / kThreads;
      int32_t hs[R], lms[R];
      Call<T> ks[R];
#pragma unroll
      for (int j = 0; j < R; ++j) {
        const int64_t x = b0 + j * kThreads + threadIdx.x;
        hs[j] = a.hd[x < a.n ? x : a.n - 1];
      }
#pragma unroll
      for (int j = 0; j < R; ++j) {
        const int64_t x = b0 + j * kThreads + threadIdx.x;
        ks[j] = call_any(a, hs[j], x < a.n ? x : a.n - 1);
        lms[j] = a.ltp[ks[j].m];
      }
#pragma unroll
      for (int j = 0; j < R; ++j)
        if (b0 + j * kThreads < a.n) round(b0 + j * kThreads, hs[j], ks[j], lms[j]);
    }
  } else {
    for (int64_t base = (int64_t)blockIdx.x * kThreads; base < a.n; base += (int64_t)gridDim.x * kThreads) {
      if (block_idle(a, base / kSpan)) continue;  // the same span block for the whole workgroup
      const int64_t xc = base + threadIdx.x < a.n ? base + threadIdx.x : a.n - 1;
      const int32_t h = a.hd[xc];
      const Call<T> k = call_any(a, h, xc);
      round(base, h, k, a.ltp[k.m]);
    }
  }
  // The next level runs while any position is in a segment of two or more
  // keys: a flag, set with plain stores.  Calls are counted per workgroup.
  if (a.sort_mode && __syncthreads_or(any_active) && threadIdx.x == 0) *a.active = 1ull;
  if (a.wcalls) {
    __shared__ unsigned long long csum;
    if (threadIdx.x == 0) csum = 0;
    __syncthreads();
    if (ncall) atomicAdd(&csum, ncall);
    __syncthreads();
    if (threadIdx.x == 0 && csum) a.wcalls[blockIdx.x] += csum;
  }
}

// Bits a .. b of a 64-bit mask (empty when b < a); 0 <= a, b <= 63 or b = -1.
__device__ __forceinline__ uint64_t bits_upto(int b) { return b < 0 ? 0ull : b >= 63 ? ~0ull : (2ull << b) - 1; }
__device__ __forceinline__ uint64_t bit_range(int a, int b) { return b < a ? 0ull : bits_upto(b) & ~bits_upto(a - 1); }

// Every remaining call on the sides filed this level (2 .. kShort keys
// each), one wave per side and one key per lane, in nxt (the level's
// output).  The wave runs the same closed form level by level on all
// sub-segments of its side at once: a lane's sub-segment is (s, len), its key
// is read from lane s, smaller-key counts come from the ballot of "smaller",
// and the q and r lanes are filed by rank in LDS to find their partners.
// The keys end where the recursion leaves them (ascending).
template <typename T>
__global__ __launch_bounds__(kThreads) void small_kernel(LevelArgs<T> a) {
  constexpr int NW = kThreads / 64;
  __shared__ int32_t qs[NW][kShort + 1], rs[NW][kShort + 1];
  __shared__ T vs[NW][kShort];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __shared__ int32_t s_end[kSmallGroups];  // inclusive prefix of the list lengths
  __shared__ int32_t s_total;
  unsigned long long ncall = 0;
  constexpr int GL = kSmallGroups / 64;  // lists per lane in the prefix
  if (w == 0) {
    int32_t c[GL], sum = 0;
#pragma unroll
    for (int q = 0; q < GL; ++q) {
      c[q] = GL * lane + q < a.ngroups ? a.nsmall[GL * lane + q] : 0;
      sum += c[q];
    }
    int32_t inc = sum;
    for (int d = 1; d < 64; d <<= 1) {
      const int32_t o = __shfl_up(inc, d);
      if (lane >= d) inc += o;
    }
    int32_t run = inc - sum;
#pragma unroll
    for (int q = 0; q < GL; ++q) {
      run += c[q];
      s_end[GL * lane + q] = run;
    }
    if (lane == 63) s_total = inc;
  }
  __syncthreads();
  const int32_t total = s_total;
  for (int32_t e = (int32_t)blockIdx.x * NW + w; e < total; e += (int32_t)gridDim.x * NW) {
    // the list holding entry e: the first whose prefix exceeds e (first the
    // lane whose last list ends past e, then among that lane's lists)
    const uint64_t past = __ballot(s_end[GL * lane + GL - 1] > e);
    int l = GL * __builtin_ctzll(past);
    while (s_end[l] <= e) ++l;
    const int32_t off = e - (l > 0 ? s_end[l - 1] : 0);
    const int2 sg = a.small[l * a.small_cap + off];
    const int64_t gl = sg.x;
    const int L = sg.y;
    T v = lane < L ? a.nxt[gl + lane] : T(0);
    int s = 0, len = lane < L ? L : 0;
    for (;;) {
      const bool act = len >= 2;
      if (!__ballot(act)) break;
      const int right = s + len - 1;
      const T key = __shfl(v, act ? s : lane);
      const bool lt = act && lane != s && !(key <= v);
      const uint64_t ltm = __ballot(lt);
      const int c = act ? __popcll(ltm & bit_range(s + 1, right)) : 0;
      const int i = s + c;
      const T vi1 = __shfl(v, act && i < right ? i + 1 : lane);
      const int m = (act && i < right && key <= vi1) ? i + 1 : i;
      const int lp = act && lane > s ? __popcll(ltm & bit_range(s + 1, lane)) : 0;
      if (act && lane != s) {
        if (lane <= m) {
          if (!lt) qs[w][s + (lane - s) - lp] = lane;  // q, by rank in (s, m]
        } else if (lt) {
          rs[w][s + (c - lp + 1)] = lane;  // r, by rank from the right in (m, right]
        }
      }
      KS_LDS_WAIT();
      int dest = lane;
      if (act) {
        const int kq = (lane - s) - lp;
        if (lane == s)
          dest = i;
        else if (lane <= m)
          dest = lt ? lane - 1 : (kq == 1 ? i + 1 : rs[w][s + kq - 1]);
        else
          dest = lt ? qs[w][s + (c - lp + 1)] - 1 : lane;
      }
      if (act && lane == s) {
        if (a.calls) {
          const unsigned long long j = atomicAdd(a.ncalls, 1ull);
          if ((int64_t)j < a.calls_cap) {
            a.calls[3 * j] = gl + s;
            a.calls[3 * j + 1] = gl + right;
            a.calls[3 * j + 2] = gl + i;
          }
        } else {
          ++ncall;
        }
      }
      vs[w][dest] = v;
      KS_LDS_WAIT();
      v = vs[w][lane < kShort ? lane : 0];
      KS_LDS_WAIT();  // all reads done before the next level's writes
      if (act) {
        if (lane < i) {
          len = c >= 2 ? c : 0;
        } else if (lane == i) {
          len = 0;
        } else {
          s = i + 1;
          len = right - i >= 2 ? right - i : 0;
        }
      }
    }
    if (lane < L) a.nxt[gl + lane] = v;
  }
  if (a.wcalls) {
    __shared__ unsigned long long csum;
    if (threadIdx.x == 0) csum = 0;
    __syncthreads();
    if (ncall) atomicAdd(&csum, ncall);
    __syncthreads();
    if (threadIdx.x == 0 && csum) a.wcalls[kPairGrid + blockIdx.x] += csum;
  }
}

// Sums the per-workgroup call counts into *out (one workgroup).
__global__ __launch_bounds__(kThreads) void sum_calls(const unsigned long long* w, int nslots, unsigned long long* out) {
  __shared__ unsigned long long part[kThreads];
  unsigned long long s = 0;
  for (int j = threadIdx.x; j < nslots; j += kThreads) s += w[j];
  part[threadIdx.x] = s;
  __syncthreads();
  for (int d = kThreads / 2; d > 0; d >>= 1) {
    if (threadIdx.x < d) part[threadIdx.x] += part[threadIdx.x + d];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out += part[0];
}

// Whole array as one segment (sort mode, n >= 2).
__global__ __launch_bounds__(kThreads) void init_whole(int32_t* hd, int32_t* ln, int64_t n) {
  for (int64_t x = (int64_t)blockIdx.x * kThreads + threadIdx.x; x < n; x += (int64_t)gridDim.x * kThreads) {
    hd[x] = 0;
    if (x == 0) ln[0] = (int32_t)n;
  }
}

__global__ __launch_bounds__(kThreads) void fill_i32(int32_t* p, int64_t n, int32_t v) {
  for (int64_t x = (int64_t)blockIdx.x * kThreads + threadIdx.x; x < n; x += (int64_t)gridDim.x * kThreads) p[x] = v;
}

// Level mode: chunk j covers positions [cs[j], cs[j] + kSpan) of segment
// (cl[j], clen[j]).
__global__ __launch_bounds__(kThreads) void mark_segments(int32_t* hd, int32_t* ln, const int64_t* cl,
                                                            const int64_t* clen, const int64_t* cs) {
  const int64_t left = cl[blockIdx.x], len = clen[blockIdx.x], s0 = cs[blockIdx.x];
  const int64_t end = min(left + len, s0 + (int64_t)kSpan);
  for (int64_t x = s0 + threadIdx.x; x < end; x += kThreads) {
    hd[x] = (int32_t)left;
    if (x == left) ln[x] = (int32_t)len;
  }
}

__global__ __launch_bounds__(kThreads) void gather_pivots(const int32_t* piv_at, const int64_t* left,
                                                            const uint8_t* ok, int64_t nseg, int64_t* out) {
  for (int64_t s = (int64_t)blockIdx.x * kThreads + threadIdx.x; s < nseg; s += (int64_t)gridDim.x * kThreads)
    if (ok[s]) out[s] = piv_at[left[s]];
}

// ------------------------------------------------------------------ host

static int grid_for(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>((n + kThreads - 1) / kThreads, kPairGrid)); }

// Device scratch of a call, laid out in two passes over the same sequence
// of take() calls: the first (no base) measures, the second hands out
// pieces of an arena of at least that size.
struct Carve {
  char* base = nullptr;
  size_t off = 0;
  template <typename P>
  int take(P** out, size_t count) {
    if (count == 0) count = 1;
    *out = base ? (P*)(base + off) : nullptr;
    off += (count * sizeof(P) + 255) & ~(size_t)255;
    return KSORT_OK;
  }
};

// Scratch kept per (device, stream) between calls and grown on demand (a
// call's own allocations and frees cost about 3 ms at 7e6 keys, as much as
// a third of the sort), with a pinned word pair for the read-backs.  The
// lock is held for a whole call.
struct Arena {
  std::mutex mu;
  void* base = nullptr;
  size_t bytes = 0;
  unsigned long long* h = nullptr;
};

static std::mutex g_arena_mu;
// never destroyed: calls may run during static destruction of the process
static auto* g_arenas = new std::map<std::pair<int, hipStream_t>, std::unique_ptr<Arena>>();

static Arena* arena_for(hipStream_t st) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  std::lock_guard<std::mutex> lk(g_arena_mu);
  auto& p = (*g_arenas)[std::make_pair(dev, st)];
  if (!p) p.reset(new Arena);
  return p.get();
}

// Makes the arena hold `need` bytes (the caller holds its lock).
static int arena_reserve(Arena& A, size_t need, hipStream_t st) {
  if (!A.h) KSORT_HIP(hipHostMalloc((void**)&A.h, 2 * sizeof(unsigned long long), hipHostMallocDefault));
  if (need <= A.bytes) return KSORT_OK;
  if (A.base) {
    KSORT_HIP(hipStreamSynchronize(st));
    KSORT_HIP(hipFree(A.base));
    A.base = nullptr;
    A.bytes = 0;
  }
  KSORT_HIP(hipMalloc(&A.base, need));
  A.bytes = need;
  return KSORT_OK;
}

// Buffers of a level; hd[1] and ln[1] (the next level's) only in sort mode.
template <typename T>
static int alloc_level(Carve& B, LevelArgs<T>& a, int64_t n, bool sort_mode, int32_t* hd[2], int32_t* ln[2]) {
  int rc = 0;
  const int64_t nb = (n + kSpan - 1) / kSpan;
  a.n = n;
  a.nblocks = (int32_t)nb;
  hd[1] = ln[1] = nullptr;
  if ((rc = B.take(&hd[0], (size_t)n)) || (rc = B.take(&ln[0], (size_t)n)) || (rc = B.take(&a.ltp, (size_t)n)) ||
      (rc = B.take(&a.qpos, (size_t)n)) || (rc = B.take(&a.rpos, (size_t)n)) || (rc = B.take(&a.qkey, (size_t)n)) ||
      (rc = B.take(&a.rkey, (size_t)n)) || (rc = B.take(&a.sstat[0], (size_t)2 * nb)) ||
      (rc = B.take(&a.sctr, 2)) || (rc = B.take(&a.err, 1)))
    return rc;
  a.sstat[1] = a.sstat[0] ? a.sstat[0] + nb : nullptr;
  a.spin_limit = spin_limit_setting();
  if (sort_mode) {
    if ((rc = B.take(&hd[1], (size_t)n)) || (rc = B.take(&ln[1], (size_t)n)) || (rc = B.take(&a.active, 1))) return rc;
  }
  a.hd = hd[0];
  a.ln = ln[0];
  a.hd2 = hd[1];
  a.ln2 = ln[1];
  return KSORT_OK;
}

// Clears the look-back words, ticket counters and error flag of a run.
template <typename T>
static int clear_scan_state(const LevelArgs<T>& a, hipStream_t st) {
  KSORT_HIP(hipMemsetAsync(a.sstat[0], 0, (size_t)2 * a.nblocks * sizeof(uint64_t), st));
  KSORT_HIP(hipMemsetAsync(a.sctr, 0, 2 * sizeof(int32_t), st));
  KSORT_HIP(hipMemsetAsync(a.err, 0, sizeof(int32_t), st));
  return KSORT_OK;
}

template <typename T>
static int launch_level(const LevelArgs<T>& a, hipStream_t st) {
  const int nb = a.nblocks;
  hipLaunchKernelGGL(scan_level<T>, dim3((nb + kScanChunk - 1) / kScanChunk), dim3(kThreads), 0, st, a);
  hipLaunchKernelGGL(move_kernel<T>, dim3(grid_for(a.n)), dim3(kThreads), 0, st, a);
  hipLaunchKernelGGL(pair_kernel<T>, dim3(grid_for(a.n)), dim3(kThreads), 0, st, a);
  if (a.small) hipLaunchKernelGGL(small_kernel<T>, dim3(kSmallGrid), dim3(kThreads), 0, st, a);
  KSORT_HIP(hipGetLastError());
  return KSORT_OK;
}

static int check_device() {
  int dev = 0;
  KSORT_HIP(hipGetDevice(&dev));
  const DeviceInfo* di = nullptr;
  int rc = device_info(dev, &di);
  if (rc) return rc;
  if (!di->gfx950) return fail(KSORT_EUNSUPPORTED, "device is " + di->arch + ", not gfx950");
  return KSORT_OK;
}

template <typename T>
static int sort_exact(T* data, int64_t n, int64_t* d_first_pivot, int64_t* d_calls, int64_t calls_cap,
                      int64_t* d_ncalls, hipStream_t st) {
  if (d_ncalls) KSORT_HIP(hipMemsetAsync(d_ncalls, 0, sizeof(int64_t), st));
  if (n <= 1) {
    if (d_first_pivot) {
      const int64_t v = n == 0 ? -1 : 0;
      KSORT_HIP(hipMemcpyAsync(d_first_pivot, &v, sizeof v, hipMemcpyHostToDevice, st));
      KSORT_HIP(hipStreamSynchronize(st));
    }
    return KSORT_OK;
  }
  Arena* A = arena_for(st);
  if (!A) return fail(KSORT_EHIP, "hipGetDevice failed");
  std::lock_guard<std::mutex> lk(A->mu);
  LevelArgs<T> a{};
  int32_t *H[2], *Ln[2];
  T* scratch = nullptr;
  uint8_t* act_ring = nullptr;  // three levels of per-block activity flags
  const bool count_per_group = d_ncalls && !d_calls;  // calls counted per workgroup, summed at the end
  // per pair_kernel workgroup: its iterations of kThreads positions, each
  // filing at most kThreads / 2 sides (disjoint, two keys or more)
  a.npair = grid_for(n);
  a.ngroups = std::min(kSmallGroups, a.npair);
  {
    // a workgroup's rounds of kThreads positions each file at most
    // kThreads / 2 sides (disjoint, two keys or more); it takes at most
    // ceil(4 * blocks / npair) units of kUnit / kThreads rounds, and a group
    // holds at most ceil(npair / ngroups) workgroups
    const int64_t nb = (n + kSpan - 1) / kSpan;
    const int64_t iters = (4 * nb + a.npair - 1) / a.npair * (kUnit / kThreads);
    a.small_cap = ((int64_t)a.npair + a.ngroups - 1) / a.ngroups * iters * (kThreads / 2) + 1;
  }
  auto layout = [&](Carve& B) {
    int r = alloc_level<T>(B, a, n, true, H, Ln);
    if (!r) r = B.take(&scratch, (size_t)n);
    if (!r) r = B.take(&act_ring, (size_t)3 * a.nblocks);
    if (!r) r = B.take(&a.small, (size_t)a.ngroups * a.small_cap);
    if (!r) r = B.take(&a.nsmall, (size_t)a.ngroups);
    if (!r) r = B.take(&a.blist[0], (size_t)2 * a.nblocks);
    if (!r) r = B.take(&a.nblist[0], 1);  // (every piece starts a 256-byte line)
    if (!r) r = B.take(&a.nblist[1], 1);
    if (!r && count_per_group) r = B.take(&a.wcalls, (size_t)(kPairGrid + kSmallGrid));
    return r;
  };
  Carve measure;
  int rc = layout(measure);
  if (rc || (rc = arena_reserve(*A, measure.off, st))) return rc;
  Carve B;
  B.base = (char*)A->base;
  if ((rc = layout(B))) return rc;
  unsigned long long* h_active = A->h;
  KSORT_HIP(hipMemsetAsync(act_ring, 1, (size_t)3 * a.nblocks, st));
  a.blist[1] = a.blist[0] + a.nblocks;
  KSORT_HIP(hipMemsetAsync(a.nblist[0], 0, sizeof(int32_t), st));
  KSORT_HIP(hipMemsetAsync(a.nblist[1], 0, sizeof(int32_t), st));
  a.sort_mode = 1;
  a.calls = d_calls;
  a.calls_cap = d_calls ? calls_cap : 0;
  a.ncalls = (unsigned long long*)d_ncalls;
  if (count_per_group)
    KSORT_HIP(hipMemsetAsync(a.wcalls, 0, (size_t)(kPairGrid + kSmallGrid) * sizeof(unsigned long long), st));
  if ((rc = clear_scan_state<T>(a, st))) return rc;
  hipLaunchKernelGGL(init_whole, dim3(grid_for(n)), dim3(kThreads), 0, st, H[0], Ln[0], n);
  KSORT_HIP(hipGetLastError());
  T* bufs[2] = {data, scratch};
  int cur = 0;
  // Levels are launched in groups between reads of the active count; a
  // level after the last one finds every block idle.  Every level ends with
  // a complete array in its output buffer (keys final for two levels are in
  // both buffers, keys final since the level before are copied once).
  // Every level ends at least one key's partitioning, so n levels suffice.
  constexpr int kGroup = 8;
  for (int64_t level = 0; level < n;) {
    const int64_t stop = std::min<int64_t>(n, level + kGroup);
    for (; level < stop; ++level) {
      a.cur = bufs[cur];
      a.nxt = bufs[cur ^ 1];
      a.hd = H[cur];
      a.ln = Ln[cur];
      a.hd2 = H[cur ^ 1];
      a.ln2 = Ln[cur ^ 1];
      a.act = act_ring + (size_t)(level % 3) * a.nblocks;
      a.act_prev = act_ring + (size_t)((level + 2) % 3) * a.nblocks;
      a.act_next = act_ring + (size_t)((level + 1) % 3) * a.nblocks;
      a.first_pivot = level == 0 ? d_first_pivot : nullptr;
      a.par = (int32_t)(level & 1);
      if ((rc = launch_level<T>(a, st))) return rc;
      cur ^= 1;
    }
    KSORT_HIP(hipMemcpyAsync(h_active, a.active, sizeof(unsigned long long), hipMemcpyDeviceToHost, st));
    KSORT_HIP(hipMemcpyAsync(h_active + 1, a.err, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    KSORT_HIP(hipStreamSynchronize(st));
    if (((const int32_t*)(h_active + 1))[0] != 0) return fail(KSORT_EINTERNAL, "a look-back wait timed out");
    if (*h_active == 0) break;
  }
  if (cur == 1) KSORT_HIP(hipMemcpyAsync(data, scratch, (size_t)n * sizeof(T), hipMemcpyDeviceToDevice, st));
  if (a.wcalls) {
    hipLaunchKernelGGL(sum_calls, dim3(1), dim3(kThreads), 0, st, a.wcalls, kPairGrid + kSmallGrid, a.ncalls);
    KSORT_HIP(hipGetLastError());
  }
  KSORT_HIP(hipStreamSynchronize(st));
  return KSORT_OK;
}

template <typename T>
static int level_exact(const T* d_in, T* d_out, int64_t n, const int64_t* d_left, const int64_t* d_len, int64_t nseg,
                       int64_t* d_pivot, hipStream_t st) {
  std::vector<int64_t> hl((size_t)nseg), hn((size_t)nseg);
  KSORT_HIP(hipMemcpyAsync(hl.data(), d_left, (size_t)nseg * sizeof(int64_t), hipMemcpyDeviceToHost, st));
  KSORT_HIP(hipMemcpyAsync(hn.data(), d_len, (size_t)nseg * sizeof(int64_t), hipMemcpyDeviceToHost, st));
  KSORT_HIP(hipStreamSynchronize(st));
  std::vector<uint8_t> ok((size_t)nseg, 0);
  std::vector<int64_t> order;
  bool bad = false;
  for (int64_t s = 0; s < nseg; ++s) {
    if (hl[s] < 0 || hn[s] < 1 || hl[s] > n - hn[s]) {
      bad = true;
      continue;
    }
    ok[s] = 1;
    order.push_back(s);
  }
  std::sort(order.begin(), order.end(), [&](int64_t x, int64_t y) { return hl[x] < hl[y]; });
  for (size_t j = 1; j < order.size(); ++j)
    if (hl[order[j]] < hl[order[j - 1]] + hn[order[j - 1]]) return fail(KSORT_EINVAL, "segments overlap");
  std::vector<int64_t> cl, clen, cs;
  for (int64_t s : order)
    for (int64_t p = hl[s]; p < hl[s] + hn[s]; p += kSpan) {
      cl.push_back(hl[s]);
      clen.push_back(hn[s]);
      cs.push_back(p);
    }
  Arena* A = arena_for(st);
  if (!A) return fail(KSORT_EHIP, "hipGetDevice failed");
  std::lock_guard<std::mutex> lk(A->mu);
  LevelArgs<T> a{};
  int32_t *H[2], *Ln[2];
  int64_t *dcl = nullptr, *dclen = nullptr, *dcs = nullptr;
  uint8_t* dok = nullptr;
  auto layout = [&](Carve& B) {
    int r = alloc_level<T>(B, a, n, false, H, Ln);
    if (!r) r = B.take(&dcl, cl.size());
    if (!r) r = B.take(&dclen, cl.size());
    if (!r) r = B.take(&dcs, cl.size());
    if (!r) r = B.take(&dok, (size_t)nseg);
    if (!r) r = B.take(&a.piv_at, (size_t)n);
    return r;
  };
  Carve measure;
  int rc = layout(measure);
  if (rc || (rc = arena_reserve(*A, measure.off, st))) return rc;
  Carve B;
  B.base = (char*)A->base;
  if ((rc = layout(B))) return rc;
  KSORT_HIP(hipMemcpyAsync(dcl, cl.data(), cl.size() * sizeof(int64_t), hipMemcpyHostToDevice, st));
  KSORT_HIP(hipMemcpyAsync(dclen, clen.data(), clen.size() * sizeof(int64_t), hipMemcpyHostToDevice, st));
  KSORT_HIP(hipMemcpyAsync(dcs, cs.data(), cs.size() * sizeof(int64_t), hipMemcpyHostToDevice, st));
  KSORT_HIP(hipMemcpyAsync(dok, ok.data(), ok.size(), hipMemcpyHostToDevice, st));
  hipLaunchKernelGGL(fill_i32, dim3(grid_for(n)), dim3(kThreads), 0, st, H[0], n, -1);
  if (!cl.empty()) hipLaunchKernelGGL(mark_segments, dim3((unsigned)cl.size()), dim3(kThreads), 0, st, H[0], Ln[0], dcl, dclen, dcs);
  KSORT_HIP(hipGetLastError());
  a.cur = d_in;
  a.nxt = d_out;
  a.sort_mode = 0;
  a.par = 0;
  if ((rc = clear_scan_state<T>(a, st))) return rc;
  if ((rc = launch_level<T>(a, st))) return rc;
  hipLaunchKernelGGL(gather_pivots, dim3(grid_for(nseg)), dim3(kThreads), 0, st, a.piv_at, d_left, dok, nseg, d_pivot);
  KSORT_HIP(hipGetLastError());
  KSORT_HIP(hipMemcpyAsync(A->h, a.err, sizeof(int32_t), hipMemcpyDeviceToHost, st));
  KSORT_HIP(hipStreamSynchronize(st));
  if (((const int32_t*)A->h)[0] != 0) return fail(KSORT_EINTERNAL, "a look-back wait timed out");
  if (bad) return fail(KSORT_EINVAL, "a segment is outside [0, n) or has len < 1");
  return KSORT_OK;
}

}  // namespace exact

void release_exact_arenas() {
  std::lock_guard<std::mutex> lk(exact::g_arena_mu);
  for (auto& kv : *exact::g_arenas) {
    exact::Arena& A = *kv.second;
    std::lock_guard<std::mutex> al(A.mu);
    if (A.base) (void)hipFree(A.base);
    if (A.h) (void)hipHostFree(A.h);
    A.base = nullptr;
    A.h = nullptr;
    A.bytes = 0;
  }
}

}  // namespace ksort

using namespace ksort;

extern "C" {

int ksort_partition_level_exact(int dtype, const void* d_in, void* d_out, int64_t n, const int64_t* d_seg_left,
                                const int64_t* d_seg_len, int64_t nseg, int64_t* d_pivot, void* stream) {
  if (dtype != KSORT_F64 && dtype != KSORT_F32) return fail(KSORT_EINVAL, "bad dtype");
  if (n < 0 || nseg < 0) return fail(KSORT_EINVAL, "negative size");
  if (n >= (int64_t)1 << 31) return fail(KSORT_EINVAL, "the exact arrangement takes n < 2^31");
  if (nseg == 0) return KSORT_OK;
  if (!d_in || !d_out || !d_seg_left || !d_seg_len || !d_pivot) return fail(KSORT_EINVAL, "null pointer");
  if (d_in == d_out) return fail(KSORT_EINVAL, "d_in and d_out must not overlap");
  int rc = exact::check_device();
  if (rc) return rc;
  hipStream_t st = (hipStream_t)stream;
  if (dtype == KSORT_F64)
    return exact::level_exact<double>((const double*)d_in, (double*)d_out, n, d_seg_left, d_seg_len, nseg, d_pivot,
                                      st);
  return exact::level_exact<float>((const float*)d_in, (float*)d_out, n, d_seg_left, d_seg_len, nseg, d_pivot, st);
}

int ksort_sort_exact(int dtype, void* d_data, int64_t n, int64_t* d_first_pivot, int64_t* d_calls,
                     int64_t calls_cap, int64_t* d_ncalls, void* stream) {
  if (dtype != KSORT_F64 && dtype != KSORT_F32) return fail(KSORT_EINVAL, "bad dtype");
  if (n < 0 || calls_cap < 0) return fail(KSORT_EINVAL, "negative size");
  if (n >= (int64_t)1 << 31) return fail(KSORT_EINVAL, "the exact arrangement takes n < 2^31");
  if (n > 0 && !d_data) return fail(KSORT_EINVAL, "null data pointer");
  if (d_calls && !d_ncalls) return fail(KSORT_EINVAL, "d_calls needs d_ncalls");
  int rc = exact::check_device();
  if (rc) return rc;
  hipStream_t st = (hipStream_t)stream;
  if (dtype == KSORT_F64)
    return exact::sort_exact<double>((double*)d_data, n, d_first_pivot, d_calls, calls_cap, d_ncalls, st);
  return exact::sort_exact<float>((float*)d_data, n, d_first_pivot, d_calls, calls_cap, d_ncalls, st);
}

}  // extern "C"
