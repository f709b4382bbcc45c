// K-sort device kernels for gfx950 (CDNA4, wave64).
//
// The paper's method (arXiv 1107.3622, Section 1.1) partitions a[left..right]
// around key = a[left]: keys that compare `key <= x` false go left of the key,
// the others right, and both sides are then treated the same way.  Step-4
// leaves the key at i = left + (number of keys smaller than it); Steps 5-6
// recurse on [left, i-1] and [i+1, right]; a side with one key is final
// (Section 1.2 note).
//
// Here every "level" of that recursion is one data-parallel pass over all
// live segments at once (the stage kernel):
//   * partition work: each live segment is cut into tiles of BLOCK*ITEMS
//     keys.  A tile classifies its keys against the segment's key with one
//     compare each, counts them with wave ballots and popcounts, scans the
//     per-wave counts in LDS, obtains the count of smaller keys in the
//     segment's earlier tiles by decoupled look-back, and scatters its keys
//     through an LDS staging buffer into two contiguous runs of the
//     ping-pong buffer: smaller keys filling [left, i-1] upward, the others
//     filling [i+1, right] downward (so no separate counting pass is needed
//     to know i).  The segment's last tile knows i, writes the key to its
//     final place in the caller's array and emits the two sides.
//   * finish work: a segment of at most CUT keys is loaded into LDS once and
//     sorted there by the same rule, level after level, then written to its
//     final place.
// Both kinds of work come from one ticket counter per stage, partition tiles
// first, so a persistent grid drains the stage without host involvement.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ksort_types.h"

namespace ksort {

constexpr int kWave = 64;

// ---------------------------------------------------------------------------
// small helpers

__device__ __forceinline__ int lane_id() { return threadIdx.x & (kWave - 1); }

__device__ __forceinline__ int mbcnt(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0));
}

template <typename I>
__device__ __forceinline__ I uniform(I v) {
  return (I)__builtin_amdgcn_readfirstlane((int)v);
}

__device__ __forceinline__ int64_t uniform64(int64_t v) {
  uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
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

// Inclusive prefix sum across the 64 lanes of a wave.
__device__ __forceinline__ int wave_inclusive_scan(int v) {
  const int lane = lane_id();
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    int u = __shfl_up(v, d, kWave);
    if (lane >= d) v += u;
  }
  return v;
}

__device__ __forceinline__ int64_t wave_sum64(int64_t v) {
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) v += __shfl_xor(v, d, kWave);
  return v;
}

// Look-back word: count in bits 0..39, flag in 40..41, epoch in 42..63.
constexpr uint64_t kFlagAgg = 1;   // tile's own count of smaller keys
constexpr uint64_t kFlagPre = 2;   // count over the segment up to and including the tile
__device__ __forceinline__ uint64_t status_word(uint32_t epoch, uint64_t flag, uint64_t count) {
  return ((uint64_t)epoch << 42) | (flag << 40) | count;
}

// Finish-list packing of an in-LDS sub-segment: start in the low 16 bits,
// length in the high 16 bits.
__device__ __forceinline__ uint32_t pack_sub(uint32_t l, uint32_t len) { return l | (len << 16); }

// ---------------------------------------------------------------------------
// shared memory layouts

template <typename T, int BLOCK, int ITEMS>
struct PartSmem {
  static constexpr int NW = BLOCK / kWave;
  T stage[BLOCK * ITEMS];
  int32_t off_lt[ITEMS * NW];
  int32_t off_ge[ITEMS * NW];
  int64_t xlt;
  int32_t tot_lt, tot_ge;
  int32_t em_slot[2], em_first[2], em_nt[2];
};

template <typename T, int BLOCK, int CUT>
struct FinSmem {
  static constexpr int NW = BLOCK / kWave;
  static constexpr int FI = CUT / BLOCK;
  T keys[CUT];
  uint32_t sub[CUT];
  uint32_t pre[CUT + 1];
  int32_t off[FI * NW];
};

template <typename T, int BLOCK, int ITEMS, int CUT>
union StageSmem {
  PartSmem<T, BLOCK, ITEMS> p;
  FinSmem<T, BLOCK, CUT> f;
};

// ---------------------------------------------------------------------------
// decoupled look-back: returns the number of smaller keys in tiles
// first_tile .. t-1 of the segment.  Executed by one whole wave.

__device__ __forceinline__ int64_t look_back(const StageArgs& a, int32_t t, int32_t first_tile) {
  const int lane = lane_id();
  int64_t excl = 0;
  int32_t j = t - 1 - lane;
  for (;;) {
    const bool in_seg = j >= first_tile;
    uint64_t w = 0;
    uint64_t flag = 0;
    if (in_seg) {
      for (;;) {
        w = ld_agent(a.status + j);
        flag = (w >> 40) & 3;
        if ((uint32_t)(w >> 42) == a.epoch && flag != 0) break;
        __builtin_amdgcn_s_sleep(1);
      }
    }
    const uint64_t pre_mask = __ballot(in_seg && flag == kFlagPre);
    int64_t c = in_seg ? (int64_t)(w & ((1ull << 40) - 1)) : 0;
    if (pre_mask) {
      const int stop = __builtin_ctzll(pre_mask);  // nearest predecessor with a full prefix
      if (lane > stop) c = 0;
      return excl + wave_sum64(c);
    }
    excl += wave_sum64(c);
    j -= kWave;
  }
}

// ---------------------------------------------------------------------------
// The last tile of a live segment: Step-4 (the key to its final index i) and
// Steps 5-6 (the two sides become segments of the next stage).  All tiles of
// the segment have published their counts, hence have read their keys, so
// the key may be written into the caller's array even when that array is
// this stage's input.
template <typename T, int TILE>
__device__ void emit_children(const StageArgs& a, int32_t* em_slot, int32_t* em_first, int32_t* em_nt,
                              int64_t left, int64_t len, int64_t total_lt, T key, int32_t root,
                              int32_t bufi, int32_t parity, const BufPair& bp) {
  const int tid = threadIdx.x;
  const int par = a.stage & 1;
  const int64_t i = left + total_lt;
  if (tid == 0) {
    ((T*)bp.data)[i] = key;
    if (root >= 0 && a.pivot_out) a.pivot_out[root] = a.pivot_relative ? total_lt : i;
    int nchild = 0;
    em_nt[0] = em_nt[1] = 0;
    if (a.emit_children) {
      StageCtr* nx = a.ctr + ((a.stage + 1) % 3);
      const int npar = par ^ 1;
      const int64_t cl[2] = {left, i + 1};
      const int64_t cn[2] = {total_lt, len - 1 - total_lt};
      uint64_t live_keys = 0, fin_keys = 0;
      for (int c = 0; c < 2; ++c) {
        if (cn[c] > a.cutoff) {
          const int32_t nt = (int32_t)((cn[c] + TILE - 1) / TILE);
          const int32_t s = add_agent(&nx->nseg, 1);
          const int32_t f = add_agent(&nx->ntiles, nt);
          if (s >= a.cap_live || f + nt > a.cap_tiles) {
            st_agent(&a.flags->overflow, 1);
            continue;
          }
          Seg* d = a.live[npar] + s;
          d->left = cl[c];
          d->len = cn[c];
          d->root = -1;
          d->buf = bufi;
          d->parity = parity ^ 1;
          d->first_tile = f;
          em_slot[c] = s;
          em_first[c] = f;
          em_nt[c] = nt;
          ++nchild;
          live_keys += (uint64_t)cn[c];
        } else if (cn[c] == 1 && parity == 1) {
          // a one-key side written into the caller's array is already final
        } else if (cn[c] >= 1) {
          const int32_t f = add_agent(&nx->nfin, 1);
          if (f >= a.cap_fin) {
            st_agent(&a.flags->overflow, 1);
            continue;
          }
          Seg* d = a.fin[npar] + f;
          d->left = cl[c];
          d->len = cn[c];
          d->root = -1;
          d->buf = bufi;
          d->parity = parity ^ 1;
          d->first_tile = 0;
          ++nchild;
          fin_keys += (uint64_t)cn[c];
        }
      }
      if (nchild > 0) atomicMax(&a.flags->last_active, a.stage + 1);
      if (a.stage_keys && a.stage + 1 < a.cap_stats) {
        if (live_keys) atomicAdd((unsigned long long*)&a.stage_keys[2 * (a.stage + 1)], live_keys);
        if (fin_keys) atomicAdd((unsigned long long*)&a.stage_keys[2 * (a.stage + 1) + 1], fin_keys);
      }
    }
    if (a.pending) {
      const int32_t old = add_agent(a.pending + bufi, nchild - 1);
      if (old + nchild - 1 == 0 && a.done_stage) st_agent(a.done_stage + bufi, a.stage);
    }
  }
  __syncthreads();
  // tile map of the live children: ticket -> live slot
  for (int c = 0; c < 2; ++c) {
    const int32_t nt = em_nt[c];
    if (nt > 0) {
      int32_t* tm = a.tilemap[par ^ 1] + em_first[c];
      const int32_t s = em_slot[c];
      for (int j = tid; j < nt; j += blockDim.x) tm[j] = s;
    }
  }
}

// ---------------------------------------------------------------------------
// partition work: one tile of one live segment

template <typename T, int BLOCK, int ITEMS, int CUT>
__device__ void partition_tile(const StageArgs& a, int32_t t, PartSmem<T, BLOCK, ITEMS>& sm) {
  constexpr int NW = BLOCK / kWave;
  constexpr int TILE = BLOCK * ITEMS;
  static_assert(ITEMS * NW <= kWave, "per-wave counts must fit one wave scan");
  const int tid = threadIdx.x, lane = lane_id(), w = tid / kWave;
  const int par = a.stage & 1;

  const int32_t slot = uniform(a.tilemap[par][t]);
  const Seg* sp = a.live[par] + slot;
  const int64_t left = uniform64(sp->left);
  const int64_t len = uniform64(sp->len);
  const int32_t root = uniform(sp->root);
  const int32_t bufi = uniform(sp->buf);
  const int32_t parity = uniform(sp->parity);
  const int32_t first_tile = uniform(sp->first_tile);
  const int32_t tidx = t - first_tile;
  const int64_t o = (int64_t)tidx * TILE;
  const int32_t cnt = (int32_t)min((int64_t)TILE, len - o);
  const BufPair bp = a.bufs[bufi];
  const T* in = (const T*)(parity ? bp.scratch : bp.data);
  T* out = (T*)(parity ? bp.data : bp.scratch);
  const T key = in[left];
  const T* src = in + left + o;

  // a1/a2: load the tile (striped: item k of thread tid is element k*BLOCK+tid)
  // and classify against the key.
  T v[ITEMS];
#pragma unroll
  for (int k = 0; k < ITEMS; ++k) {
    const int e = k * BLOCK + tid;
    v[k] = (e < cnt) ? src[e] : T(0);
  }
  int rk[ITEMS];
  uint32_t is_lt = 0, is_valid = 0;
#pragma unroll
  for (int k = 0; k < ITEMS; ++k) {
    const int e = k * BLOCK + tid;
    const bool valid = e < cnt && !(tidx == 0 && e == 0);
    const bool lt = valid && !(key <= v[k]);
    const bool ge = valid && !lt;
    const uint64_t bl = __ballot(lt);
    const uint64_t bg = __ballot(ge);
    rk[k] = lt ? mbcnt(bl) : mbcnt(bg);
    is_lt |= (uint32_t)lt << k;
    is_valid |= (uint32_t)valid << k;
    if (lane == 0) {
      sm.off_lt[k * NW + w] = __popcll(bl);
      sm.off_ge[k * NW + w] = __popcll(bg);
    }
  }
  __syncthreads();

  // a3 (local part): exclusive scan of the per-(item, wave) counts, in element
  // order; publish this tile's count for the look-back.
  if (w == 0) {
    const int n = ITEMS * NW;
    const int cl = lane < n ? sm.off_lt[lane] : 0;
    const int cg = lane < n ? sm.off_ge[lane] : 0;
    const int il = wave_inclusive_scan(cl);
    const int ig = wave_inclusive_scan(cg);
    if (lane < n) {
      sm.off_lt[lane] = il - cl;
      sm.off_ge[lane] = ig - cg;
    }
    const int tot_lt = __shfl(il, kWave - 1, kWave);
    const int tot_ge = __shfl(ig, kWave - 1, kWave);
    if (lane == 0) {
      sm.tot_lt = tot_lt;
      sm.tot_ge = tot_ge;
      st_agent(a.status + t, status_word(a.epoch, tidx == 0 ? kFlagPre : kFlagAgg, (uint64_t)tot_lt));
    }
  }
  __syncthreads();

  // a4 (local part): stage the tile in LDS as [smaller keys | larger-or-equal
  // keys in reverse rank order], so that each side leaves as one contiguous run.
  const int tot_lt = sm.tot_lt, tot_ge = sm.tot_ge;
#pragma unroll
  for (int k = 0; k < ITEMS; ++k) {
    if (is_valid & (1u << k)) {
      const bool lt = is_lt & (1u << k);
      const int r = (lt ? sm.off_lt[k * NW + w] : sm.off_ge[k * NW + w]) + rk[k];
      sm.stage[lt ? r : tot_lt + (tot_ge - 1 - r)] = v[k];
    }
  }
  // a3 (global part): smaller keys in the segment's earlier tiles.
  if (w == 0) {
    int64_t xlt = 0;
    if (tidx > 0) {
      xlt = look_back(a, t, first_tile);
      if (lane == 0) st_agent(a.status + t, status_word(a.epoch, kFlagPre, (uint64_t)(xlt + tot_lt)));
    }
    if (lane == 0) sm.xlt = xlt;
  }
  __syncthreads();

  // a4: write both runs.  Smaller keys fill [left, i-1] upward, the others
  // fill [i+1, right] downward.  The runs always lie inside the segment; the
  // check below only guards the device against a corrupted count.
  const int64_t xlt = sm.xlt;
  const int64_t xge = o - (tidx > 0 ? 1 : 0) - xlt;
  const int64_t right = left + len - 1;
  if (xlt < 0 || xge < 0 || xlt + tot_lt > len - 1 || xge + tot_ge > len - 1) {
    if (tid == 0) st_agent(&a.flags->overflow, 2);
    return;
  }
  T* dlt = out + left + xlt;
  T* dge = out + (right - xge - tot_ge + 1);
  for (int s = tid; s < tot_lt + tot_ge; s += BLOCK) {
    const T x = sm.stage[s];
    if (s < tot_lt)
      dlt[s] = x;
    else
      dge[s - tot_lt] = x;
  }

  // a5/a6: the segment's last tile places the key and emits the two sides.
  if (o + cnt == len) {
    const int64_t total_lt = xlt + tot_lt;
    emit_children<T, TILE>(a, sm.em_slot, sm.em_first, sm.em_nt, left, len, total_lt, key, root, bufi,
                           parity, bp);
  }
}

// ---------------------------------------------------------------------------
// finish work: a segment of 1..CUT keys sorted in LDS by the same rule
// (first key of each sub-segment is its key; smaller keys left, the others
// right), one level per iteration, then written to the caller's array.

template <typename T, int BLOCK, int CUT>
__device__ void finish_segment(const StageArgs& a, int32_t f, FinSmem<T, BLOCK, CUT>& sm) {
  constexpr int NW = BLOCK / kWave;
  constexpr int FI = CUT / BLOCK;
  static_assert(CUT % BLOCK == 0, "cutoff must be a multiple of the block size");
  static_assert(FI * NW <= kWave, "per-wave counts must fit one wave scan");
  const int tid = threadIdx.x, lane = lane_id(), w = tid / kWave;
  const int par = a.stage & 1;

  const Seg* sp = a.fin[par] + f;
  const int64_t left = uniform64(sp->left);
  const int32_t len = uniform((int32_t)sp->len);
  const int32_t root = uniform(sp->root);
  const int32_t bufi = uniform(sp->buf);
  const int32_t parity = uniform(sp->parity);
  const BufPair bp = a.bufs[bufi];
  const T* src = (const T*)(parity ? bp.scratch : bp.data) + left;
  T* dst = (T*)bp.data + left;
  const int rows = (len + BLOCK - 1) / BLOCK;
  if (len < 1 || len > CUT) {  // never produced by the emitters; guards the LDS arrays
    if (tid == 0) st_agent(&a.flags->overflow, 3);
    return;
  }

  if (len == 1) {
    if (tid == 0) {
      if (parity) dst[0] = src[0];
      if (root >= 0 && a.pivot_out) a.pivot_out[root] = a.pivot_relative ? 0 : left;
    }
  } else {
    for (int k = 0; k < FI; ++k) {
      const int x = k * BLOCK + tid;
      if (x < len) {
        sm.keys[x] = src[x];
        sm.sub[x] = pack_sub(0, (uint32_t)len);
      }
    }
    __syncthreads();
    bool first = true;
    // every level finishes at least one key of each active sub-segment, so
    // len - 1 levels always suffice; the cap only guards against a hang
    for (int level = 0;; ++level) {
      if (level >= len) {
        if (tid == 0) st_agent(&a.flags->overflow, 4);
        break;
      }
      T val[FI];
      uint32_t sub[FI];
      int pre[FI];
      uint32_t flg = 0;
#pragma unroll
      for (int k = 0; k < FI; ++k) {
        if (k >= rows) break;
        const int x = k * BLOCK + tid;
        bool fl = false;
        if (x < len) {
          sub[k] = sm.sub[x];
          const uint32_t l = sub[k] & 0xffff, L = sub[k] >> 16;
          val[k] = sm.keys[x];
          if (L >= 2 && (uint32_t)x != l) {
            const T key = sm.keys[l];
            fl = !(key <= val[k]);
          }
        }
        const uint64_t m = __ballot(fl);
        pre[k] = mbcnt(m);
        flg |= (uint32_t)fl << k;
        if (lane == 0) sm.off[k * NW + w] = __popcll(m);
      }
      __syncthreads();
      if (w == 0) {
        const int n = rows * NW;
        const int c = lane < n ? sm.off[lane] : 0;
        const int inc = wave_inclusive_scan(c);
        if (lane < n) sm.off[lane] = inc - c;
        if (lane == kWave - 1) sm.pre[len] = (uint32_t)inc;
      }
      __syncthreads();
#pragma unroll
      for (int k = 0; k < FI; ++k) {
        if (k >= rows) break;
        const int x = k * BLOCK + tid;
        pre[k] += sm.off[k * NW + w];
        if (x < len) sm.pre[x] = (uint32_t)pre[k];
      }
      __syncthreads();
      int dest[FI];
      uint32_t nsub[FI];
      int more = 0;
#pragma unroll
      for (int k = 0; k < FI; ++k) {
        if (k >= rows) break;
        const int x = k * BLOCK + tid;
        if (x < len) {
          const uint32_t l = sub[k] & 0xffff, L = sub[k] >> 16;
          dest[k] = x;
          nsub[k] = sub[k];
          if (L >= 2) {
            const int base = (int)sm.pre[l];
            const int tot = (int)sm.pre[l + L] - base;  // smaller keys in the sub-segment
            if ((uint32_t)x == l) {
              dest[k] = (int)l + tot;
              nsub[k] = pack_sub((uint32_t)dest[k], 1);
              if (first && root >= 0 && a.pivot_out)
                a.pivot_out[root] = a.pivot_relative ? tot : left + tot;
            } else if (flg & (1u << k)) {
              dest[k] = (int)l + (pre[k] - base);
              nsub[k] = pack_sub(l, (uint32_t)tot);
            } else {
              const int rge = (x - (int)l - 1) - (pre[k] - base);
              dest[k] = (int)l + tot + 1 + rge;
              nsub[k] = pack_sub(l + (uint32_t)tot + 1, L - (uint32_t)tot - 1);
            }
            more |= (nsub[k] >> 16) >= 2;
          }
        }
      }
      __syncthreads();
#pragma unroll
      for (int k = 0; k < FI; ++k) {
        if (k >= rows) break;
        const int x = k * BLOCK + tid;
        if (x < len) {
          sm.keys[dest[k]] = val[k];
          sm.sub[dest[k]] = nsub[k];
        }
      }
      first = false;
      if (!__syncthreads_or(more)) break;
    }
    for (int k = 0; k < FI; ++k) {
      const int x = k * BLOCK + tid;
      if (x < len) dst[x] = sm.keys[x];
    }
  }
  if (tid == 0) {
    if (a.pending) {
      const int32_t old = add_agent(a.pending + bufi, -1);
      if (old - 1 == 0 && a.done_stage) st_agent(a.done_stage + bufi, a.stage);
    }
  }
}

// ---------------------------------------------------------------------------
// the stage kernel: a persistent grid drains the stage's tickets

template <typename T, int BLOCK, int ITEMS, int CUT>
__global__ __launch_bounds__(BLOCK) void stage_kernel(StageArgs a) {
  __shared__ StageSmem<T, BLOCK, ITEMS, CUT> sm;
  __shared__ int32_t s_ticket;
  StageCtr* cur = a.ctr + (a.stage % 3);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    StageCtr* nn = a.ctr + ((a.stage + 2) % 3);
    st_agent(&nn->nseg, 0);
    st_agent(&nn->ntiles, 0);
    st_agent(&nn->nfin, 0);
    st_agent(&nn->ticket, 0);
  }
  // after a capacity overflow the lists are incomplete: do nothing (the host
  // reports the error)
  if (ld_agent(&a.flags->overflow) != 0) return;
  const int32_t ntiles = uniform(min(ld_agent(&cur->ntiles), a.cap_tiles));
  const int32_t nfin = uniform(min(ld_agent(&cur->nfin), a.cap_fin));
  const int32_t nwork = ntiles + nfin;
  for (;;) {
    if (threadIdx.x == 0) s_ticket = add_agent(&cur->ticket, 1);
    __syncthreads();
    const int32_t t = uniform(s_ticket);
    if (t >= nwork) break;
    if (t < ntiles)
      partition_tile<T, BLOCK, ITEMS, CUT>(a, t, sm.p);
    else
      finish_segment<T, BLOCK, CUT>(a, t - ntiles, sm.f);
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

// Clears counters and flags before a run.
__global__ void reset_kernel(StageCtr* ctr, Flags* flags, int64_t* stage_keys, int32_t cap_stats) {
  const int tid = threadIdx.x;
  if (tid < 3) {
    ctr[tid].nseg = 0;
    ctr[tid].ntiles = 0;
    ctr[tid].nfin = 0;
    ctr[tid].ticket = 0;
  }
  if (tid == 0) {
    flags->last_active = -1;
    flags->err = 0;
    flags->overflow = 0;
  }
  if (stage_keys)
    for (int j = tid; j < 2 * cap_stats; j += blockDim.x) stage_keys[j] = 0;
}

// One block per input array (or per segment in single-level mode): validate,
// classify into the stage-0 live or finish list, and write the tile map.
__global__ void init_kernel(InitArgs ia) {
  __shared__ int32_t s_slot, s_first, s_nt;
  const StageArgs& a = ia.sa;
  const int64_t u = blockIdx.x;
  const int tid = threadIdx.x;
  if (u == 0 && tid == 0) {
    BufPair* bp = (BufPair*)a.bufs + ia.buf;
    *bp = ia.pair;
  }
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
  // the arrays join the lists of stage a.stage (0 for a fresh run; the
  // server admits requests into its current stage)
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
    if (len == 0) {
      if (a.pivot_out) a.pivot_out[root] = -1;
    } else if (!ia.level_mode && len <= a.cutoff) {
      const int32_t f = add_agent(&c0->nfin, 1);
      if (f < a.cap_fin) {
        Seg* d = a.fin[par] + f;
        d->left = left;
        d->len = len;
        d->root = root;
        d->buf = ia.buf;
        d->parity = 0;
        d->first_tile = 0;
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
        Seg* d = a.live[par] + s;
        d->left = left;
        d->len = len;
        d->root = root;
        d->buf = ia.buf;
        d->parity = ia.level_mode ? 1 : 0;
        d->first_tile = f;
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
