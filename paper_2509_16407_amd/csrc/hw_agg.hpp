// Merging duplicate keys of a write batch before they reach the table.
//
// A skewed batch (Zipf keys, as in the paper's YCSB-style and caching
// workloads, Sections 6.6 and 6.8) puts a large share of its upserts on a few
// keys.  Every upsert of a present key is an atomic on that key's value word,
// and one address serves ~80 M atomics/s on MI355X, so a single hot key can
// take longer than the rest of the batch.  With aggregation a wave takes its
// operations in windows of AGG_WIN, merges equal keys in a small LDS hash table
// (sum, min or max of their values; for insert-if-unique the first value), runs
// ONE table operation per distinct key, and gives every operation a status that
// matches one serialisation of the window: each key's first operation goes
// first, the others follow it.  Those report EXISTED (or the first one's FULL).
// REPLACE is never merged: its result depends on the order.  A key met more than
// once in a window is likely hot; in tables with hot-key accumulators its one
// operation combines into those (Ops::hot_add), in the row the caller chose.
//
// Everything here is per wave: the LDS region belongs to one wave and the
// phases are separated by wave-level fences only, so waves of a block may run
// different numbers of windows (the persistent multi-table kernel does).
#pragma once

#include "hw_ops.hpp"

namespace hw {

constexpr int AGG_WIN = 128;         // operations per window (two per lane)
constexpr int AGG_NE = 2 * AGG_WIN;  // LDS hash-table entries per wave (a power of two)
static_assert((AGG_NE & (AGG_NE - 1)) == 0 && AGG_WIN == 128, "window layout");

template <typename K>
struct AggLds {
  K key[AGG_NE];
  K val[AGG_NE];
  uint16_t lead[AGG_NE];  // window index of the entry's first operation
  uint16_t list[AGG_NE];  // compacted indices of the used entries
  uint8_t stat[AGG_NE];   // 1 if the entry merged several operations; then its table status
};

__device__ __forceinline__ bool agg_merges(int combine) {
  return combine == C_SUM || combine == C_KEEP || combine == C_MIN || combine == C_MAX;
}

// Orders this wave's LDS accesses before the ones after it (all lanes).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <typename K>
__device__ __forceinline__ K agg_identity(int combine) {
  return combine == C_MIN ? (K)~(K)0 : (K)0;
}

// Applies ops [i0, i0 + n) of `keys`/`vals` (n <= AGG_WIN, the same combine for
// all) to the table through the merge table L.  Writes status[i] if non-null.
// `row` < HOT_ROWS picks the hot-key accumulator row.  Called by all 64 lanes of
// the wave together.
template <class C>
__device__ void agg_window(const TableDev& tv, AggLds<typename C::K>& L, const typename C::K* __restrict__ keys,
                           const typename C::K* __restrict__ vals, uint64_t i0, uint32_t n, int combine,
                           uint8_t* __restrict__ status, uint32_t row) {
  using K = typename C::K;
  const uint32_t lane = __lane_id();
  const K ident = agg_identity<K>(combine);
  for (uint32_t e = lane; e < AGG_NE; e += 64) {
    L.key[e] = Keys<K>::EMPTY;
    L.val[e] = ident;
    L.stat[e] = 0;
  }
  wave_sync();
  // Phase 1: find or create each operation's entry and merge its value.
  int32_t ent[AGG_WIN / 64];
#pragma unroll
  for (int r = 0; r < AGG_WIN / 64; ++r) {
    const uint32_t w = lane + 64u * r;
    ent[r] = -1;
    if (w >= n) continue;
    const K k = keys[i0 + w];
    if (k >= Keys<K>::FIRST_INVALID) continue;  // reserved pattern: rejected below
    const K v = vals[i0 + w];
    uint32_t h = (uint32_t)fmix64((uint64_t)k) & (AGG_NE - 1);
    while (true) {
      K cur = L.key[h];
      if (cur == Keys<K>::EMPTY) {
        cur = Keys<K>::EMPTY;
        __hip_atomic_compare_exchange_strong(&L.key[h], &cur, k, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_WAVEFRONT);
        if (cur == Keys<K>::EMPTY) {
          L.lead[h] = (uint16_t)w;
          if (combine == C_KEEP) L.val[h] = v;
          break;
        }
      }
      if (cur == k) {
        L.stat[h] = 1;  // a second operation on the key
        break;
      }
      h = (h + 1) & (AGG_NE - 1);
    }
    ent[r] = (int32_t)h;
    if (combine == C_SUM) __hip_atomic_fetch_add(&L.val[h], v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
    else if (combine == C_MIN) __hip_atomic_fetch_min(&L.val[h], v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
    else if (combine == C_MAX) __hip_atomic_fetch_max(&L.val[h], v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
  }
  wave_sync();
  // Phase 2: list the used entries, then one table operation per entry.
  uint32_t n_u = 0;
  for (uint32_t base = 0; base < AGG_NE; base += 64) {
    const bool used = L.key[base + lane] != Keys<K>::EMPTY;
    const uint64_t m = __ballot(used);
    if (used) L.list[n_u + __popcll(m & ((1ull << lane) - 1))] = (uint16_t)(base + lane);
    n_u += (uint32_t)__popcll(m);
  }
  wave_sync();
  const Tile<C::T> tile;
  for (uint32_t u = lane / C::T; u < n_u; u += 64 / C::T) {
    const uint32_t e = L.list[u];
    const uint8_t st = Ops<C>::upsert(tv, tile, L.key[e], L.val[e], combine, L.stat[e] ? (int)row : -1);
    if (tile.leader()) L.stat[e] = st;
  }
  wave_sync();
  // Phase 3: every operation's status.
#pragma unroll
  for (int r = 0; r < AGG_WIN / 64; ++r) {
    const uint32_t w = lane + 64u * r;
    if (w >= n) continue;
    uint8_t st = ST_INVALID;
    if (ent[r] >= 0) {
      const uint8_t s0 = L.stat[ent[r]];
      st = L.lead[ent[r]] == w ? s0 : ((s0 == ST_DONE || s0 == ST_EXISTED) ? (uint8_t)ST_EXISTED : s0);
    }
    if (status) status[i0 + w] = st;
  }
  wave_sync();
}

}  // namespace hw
