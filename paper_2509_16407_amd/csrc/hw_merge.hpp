// Merging the upserts of a whole mixed call by key (tables created with
// HWAVE_F_MERGE_MIXED).
//
// Every upsert of a key must hold the lock of the key's primary bucket (Section
// 4.1), so a skewed batch -- Zipf keys, as in the paper's YCSB-style and caching
// workloads (Sections 6.6 and 6.8) -- puts thousands of upserts of its hottest key
// in one lock queue, one critical section after another.  The operations of a
// call are concurrent (any serialisation is a correct result), so a call may
// apply all upserts of a key back to back, as ONE table upsert of their combined
// value.  Three launches over each chunk of at most MERGE_CHUNK operations:
//
//  1. k_merge_build: each block merges the upserts of 4096 operations in an LDS
//     hash table (sum, maximum, or maximum of complements for the minimum), then
//     folds every LDS entry into a global merge table keyed by key: one atomic
//     combine per key and block.  The entry's leader is the smallest operation
//     index among its upserts (kept as chunk - index under an atomic maximum, so
//     that an empty entry is all zero).  Each upsert records its entry.
//  2. the mixed kernel (mixed_op with a workspace): the leader of an entry runs
//     one table upsert with the combined value and keeps the status in the entry;
//     the other upserts of the key (followers) skip the table and mark themselves.
//  3. k_merge_finish: followers report EXISTED (the leader went first, so the key
//     was present) or the leader's FULL / INVALID / TIMEOUT; leaders return their
//     entries to empty for the next chunk.
//
// This is the serialisation "each key's upserts consecutively, its smallest index
// first": the leader reports INSERTED when the key was absent, the followers
// EXISTED, and the value is combine(stored, v_1, ..., v_m).  KEEP (insert if
// unique) merges to the leader's value.  REPLACE is never merged: the caller
// runs it unmerged.
#pragma once

#include "hw_ops.hpp"

namespace hw {

constexpr uint32_t MERGE_CHUNK = 1u << 20;        // operations per pass (library workspace)
constexpr uint32_t MERGE_NONE = 0xFFFFFFFFu;      // op_ent of an operation that is not merged
constexpr uint32_t MERGE_FOLLOWER = 0x80000000u;  // op_ent flag set by a follower in pass 2
constexpr int MERGE_BLOCK_OPS = 4096;             // operations per block window of pass 1
constexpr int MERGE_THREADS = 1024;               // threads per block of pass 1 (16 waves: latency hiding)
constexpr int MERGE_LDS = 2048;                   // LDS entries per block (upserts <= 30% of 4096 in
                                                  // mixed batches; more spill to the global table)

struct MergeEntry {
  uint64_t acc;   // combined value: sum, maximum, or maximum of complements (minimum)
  uint32_t lead;  // chunk - (smallest operation index of the key's upserts); 0: none
  uint32_t stat;  // the leader's table status
};

// A merge workspace: `ne` (a power of two, at least twice the chunk's operations)
// entries and one word per operation.  All zero when empty (the key word holds
// key + 1, which reserved patterns aside is never 0), so it sits in the part of
// the table that clearing zero-fills.
struct MergeWs {
  uint64_t* key;     // key + 1, 0: free
  MergeEntry* ent;
  uint32_t* op_ent;  // per operation of the chunk: entry index, MERGE_NONE, | MERGE_FOLLOWER
  uint32_t ne_mask;
  uint32_t chunk;    // most operations per pass
};

__device__ __forceinline__ uint32_t merge_lead_code(const MergeWs& ws, uint64_t i) { return ws.chunk - (uint32_t)i; }

constexpr uint64_t MERGE_SALT = 0x3c6ef372fe94f82bull;

// The value an upsert contributes to its entry: the minimum is kept as the
// maximum of complements so that every combine starts from 0.
template <typename K>
__device__ __forceinline__ uint64_t merge_in(K v, int combine) {
  return combine == C_MIN ? (uint64_t)(K)~v : (uint64_t)v;
}
template <typename K>
__device__ __forceinline__ K merge_out(uint64_t acc, int combine) {
  return combine == C_MIN ? (K)~(K)acc : (K)acc;
}

__device__ __forceinline__ void merge_combine_global(uint64_t* p, uint64_t v, int combine) {
  if (combine == C_SUM) __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  else if (combine == C_MAX || combine == C_MIN)
    __hip_atomic_fetch_max(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void merge_combine_lds(uint64_t* p, uint64_t v, int combine) {
  if (combine == C_SUM) __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  else if (combine == C_MAX || combine == C_MIN)
    __hip_atomic_fetch_max(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// The global entry of key k, claimed if new (open addressing, linear probing).
// The table holds at least twice as many entries as a chunk has operations, so
// the probe always ends.
__device__ __forceinline__ uint32_t merge_slot(const MergeWs& ws, uint64_t k) {
  const uint64_t k1 = k + 1;
  uint32_t h = (uint32_t)fmix64(k ^ MERGE_SALT) & ws.ne_mask;
  while (true) {
    const uint64_t cur = cas(ws.key + h, (uint64_t)0, k1);  // returns 0 when we claimed it
    if (cur == 0 || cur == k1) return h;
    h = (h + 1) & ws.ne_mask;
  }
}

// Pass 1 over ops [0, n) (n <= ws.chunk): upserts (ops[i] == OP_UPSERT, valid key)
// are merged; op_ent receives each operation's entry or MERGE_NONE.
template <typename K>
__global__ void __launch_bounds__(MERGE_THREADS)
k_merge_build(MergeWs ws, const uint8_t* __restrict__ ops, const K* __restrict__ keys,
              const K* __restrict__ vals, uint64_t n, int combine) {
  __shared__ uint64_t lkey[MERGE_LDS];
  __shared__ uint64_t lacc[MERGE_LDS];
  __shared__ uint32_t llead[MERGE_LDS];
  __shared__ uint32_t lgent[MERGE_LDS];
  constexpr int PER = MERGE_BLOCK_OPS / MERGE_THREADS;
  const uint32_t tid = threadIdx.x;
  for (uint64_t c0 = (uint64_t)blockIdx.x * MERGE_BLOCK_OPS; c0 < n; c0 += (uint64_t)gridDim.x * MERGE_BLOCK_OPS) {
    for (uint32_t e = tid; e < MERGE_LDS; e += MERGE_THREADS) {
      lkey[e] = ~0ull;
      lacc[e] = 0;
      llead[e] = 0;
    }
    __syncthreads();
    // each operation: its LDS entry, or -2 when the LDS table had no room (then
    // it goes straight to the global table), or -1 when not merged
    int32_t le[PER];
#pragma unroll
    for (int r = 0; r < PER; ++r) {
      const uint64_t i = c0 + (uint64_t)r * MERGE_THREADS + tid;
      le[r] = -1;
      if (i >= n || ops[i] != OP_UPSERT) continue;
      const K kk = keys[i];
      if (kk >= Keys<K>::FIRST_INVALID) continue;
      const uint64_t k = (uint64_t)kk;
      const uint64_t v = merge_in<K>(vals[i], combine);
      uint32_t h = (uint32_t)fmix64(k ^ MERGE_SALT) & (MERGE_LDS - 1);
      int32_t got = -2;
      for (int p = 0; p < 32; ++p, h = (h + 1) & (MERGE_LDS - 1)) {
        uint64_t cur = lkey[h];
        if (cur == ~0ull) {
          cur = ~0ull;
          __hip_atomic_compare_exchange_strong(&lkey[h], &cur, k, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_WORKGROUP);
        }
        if (cur == ~0ull || cur == k) {
          got = (int32_t)h;
          break;
        }
      }
      le[r] = got;
      if (got >= 0) {
        merge_combine_lds(&lacc[got], v, combine);
        __hip_atomic_fetch_max(&llead[got], merge_lead_code(ws, i), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      } else {
        // no room in LDS: straight into the global table
        const uint32_t g = merge_slot(ws, k);
        merge_combine_global(&ws.ent[g].acc, v, combine);
        __hip_atomic_fetch_max(&ws.ent[g].lead, merge_lead_code(ws, i), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        ws.op_ent[i] = g;
      }
    }
    __syncthreads();
    for (uint32_t e = tid; e < MERGE_LDS; e += MERGE_THREADS) {
      const uint64_t k = lkey[e];
      if (k == ~0ull) continue;
      const uint32_t g = merge_slot(ws, k);
      lgent[e] = g;
      merge_combine_global(&ws.ent[g].acc, lacc[e], combine);
      __hip_atomic_fetch_max(&ws.ent[g].lead, llead[e], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
    // an operation that did not lead its key in this block follows for sure:
    // marked now, it skips the merge table in pass 2
#pragma unroll
    for (int r = 0; r < PER; ++r) {
      const uint64_t i = c0 + (uint64_t)r * MERGE_THREADS + tid;
      if (i >= n || le[r] == -2) continue;
      uint32_t v = MERGE_NONE;
      if (le[r] >= 0) v = lgent[le[r]] | (llead[le[r]] == merge_lead_code(ws, i) ? 0u : MERGE_FOLLOWER);
      ws.op_ent[i] = v;
    }
    __syncthreads();
  }
}

// Pass 2 helper, called for an upsert by every lane of its tile with the
// operation's op_ent word e: whether this operation runs its table upsert, and
// with which value.  A follower marks itself (leader lane) and does not touch
// the table.
template <typename K, int T>
__device__ __forceinline__ bool merge_take(const MergeWs& ws, const Tile<T>& tile, uint64_t j, uint32_t e,
                                           int combine, K* val) {
  if (e == MERGE_NONE) return true;      // not merged (invalid key): the table op reports it
  if (e & MERGE_FOLLOWER) return false;  // marked in pass 1
  const MergeEntry m = ws.ent[e];
  if (m.lead != merge_lead_code(ws, j)) {
    if (tile.leader()) ws.op_ent[j] = e | MERGE_FOLLOWER;
    return false;
  }
  if (combine != C_KEEP) *val = merge_out<K>(m.acc, combine);
  return true;
}

// Pass 3 over ops [0, n): followers take their status from the leader's, leaders
// empty their entries.  (A template, like every kernel in these headers, so that
// each translation unit's instance is mergeable at link time.)
template <typename K>
__global__ void __launch_bounds__(256)
k_merge_finish(MergeWs ws, const uint8_t* __restrict__ ops, uint64_t n, uint8_t* __restrict__ status) {
  for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (uint64_t)gridDim.x * 256) {
    if (ops[i] != OP_UPSERT) continue;
    const uint32_t e = ws.op_ent[i];
    if (e == MERGE_NONE) continue;
    if (e & MERGE_FOLLOWER) {
      const uint32_t s = ws.ent[e & ~MERGE_FOLLOWER].stat;
      if (status) status[i] = (uint8_t)((s == ST_DONE || s == ST_EXISTED) ? ST_EXISTED : s);
    } else {
      ws.key[e] = 0;
      ws.ent[e].acc = 0;
      ws.ent[e].lead = 0;
    }
  }
}

}  // namespace hw
