// Bulk kernels and their host launchers, one template instance per
// (key width, design, bucket slots, tile lanes).
//
// Each kernel maps one operation to one tile; tiles of a wave take consecutive
// operations, so the op-batch reads and status writes are coalesced.  A
// grid-stride loop keeps the grid near full occupancy for any batch size.
#pragma once

#include <hip/hip_runtime.h>

#include "hw_agg.hpp"
#include "hw_merge.hpp"
#include "hw_ops.hpp"

namespace hw {

template <class C>
__global__ void __launch_bounds__(BLOCK)
k_upsert(TableDev tv, const typename C::K* __restrict__ keys, const typename C::K* __restrict__ vals,
         uint64_t n, int combine, uint8_t* __restrict__ status) {
  using K = typename C::K;
  const Tile<C::T> tile;
  const uint64_t stride = (uint64_t)gridDim.x * (BLOCK / C::T);
  for (uint64_t i = ((uint64_t)blockIdx.x * BLOCK + threadIdx.x) / C::T; i < n; i += stride) {
    const K key = keys[i];
    const K val = vals[i];
    const uint8_t st = Ops<C>::upsert(tv, tile, key, val, combine);
    if (status && tile.leader()) status[i] = st;
  }
}

// Upsert with duplicate keys merged per wave window first (hw_agg.hpp).
template <class C>
__global__ void __launch_bounds__(BLOCK)
k_upsert_agg(TableDev tv, const typename C::K* __restrict__ keys, const typename C::K* __restrict__ vals,
             uint64_t n, int combine, uint8_t* __restrict__ status) {
  __shared__ AggLds<typename C::K> lds[BLOCK / 64];
  AggLds<typename C::K>& L = lds[threadIdx.x / 64];
  const uint64_t wave = ((uint64_t)blockIdx.x * BLOCK + threadIdx.x) / 64;
  const uint64_t n_waves = (uint64_t)gridDim.x * (BLOCK / 64);
  for (uint64_t i0 = wave * AGG_WIN; i0 < n; i0 += n_waves * AGG_WIN) {
    const uint64_t left = n - i0;
    agg_window<C>(tv, L, keys, vals, i0, (uint32_t)(left < AGG_WIN ? left : AGG_WIN), combine, status,
                  (uint32_t)(wave % HOT_ROWS));
  }
}

// Folds hot-key accumulator i into its slot's value word and frees the entry.
// Runs after the launch that filled the accumulators, in stream order.
template <typename K>
__device__ __forceinline__ void hot_flush_entry(const TableDev& tv, uint32_t i) {
  const uint64_t tagged = ld(tv.hot_tag + i);
  if (tagged == 0) return;
  const uint64_t a = ld(tv.hot_acc + i);
  K* vp = (K*)tv.slots + 2 * ((tagged & ((1ull << 56) - 1)) - 1) + 1;
  const int combine = (int)(tagged >> 56);
  if (combine == C_SUM) __hip_atomic_fetch_add(vp, (K)a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  else if (combine == C_MAX) __hip_atomic_fetch_max(vp, (K)a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  else __hip_atomic_fetch_min(vp, (K)~(K)a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  st(tv.hot_acc + i, (uint64_t)0);
  st(tv.hot_tag + i, (uint64_t)0);
}

template <typename K>
__global__ void __launch_bounds__(BLOCK) k_hot_flush(TableDev tv) {
  const uint32_t i = blockIdx.x * BLOCK + threadIdx.x;
  if (i < HOT_N) hot_flush_entry<K>(tv, i);
}

template <class C>
__global__ void __launch_bounds__(BLOCK)
k_query(TableDev tv, const typename C::K* __restrict__ keys, uint64_t n, typename C::K* __restrict__ out,
        uint8_t* __restrict__ found) {
  using K = typename C::K;
  const Tile<C::T> tile;
  const uint64_t stride = (uint64_t)gridDim.x * (BLOCK / C::T);
  for (uint64_t i = ((uint64_t)blockIdx.x * BLOCK + threadIdx.x) / C::T; i < n; i += stride) {
    K v;
    const uint8_t st = Ops<C>::query(tv, tile, keys[i], &v);
    if (tile.leader()) {
      if (out) out[i] = v;
      if (found) found[i] = st;
    }
  }
}

template <class C>
__global__ void __launch_bounds__(BLOCK)
k_erase(TableDev tv, const typename C::K* __restrict__ keys, uint64_t n, uint8_t* __restrict__ found) {
  const Tile<C::T> tile;
  const uint64_t stride = (uint64_t)gridDim.x * (BLOCK / C::T);
  for (uint64_t i = ((uint64_t)blockIdx.x * BLOCK + threadIdx.x) / C::T; i < n; i += stride) {
    const uint8_t st = Ops<C>::erase(tv, tile, keys[i]);
    if (found && tile.leader()) found[i] = st;
  }
}

// One operation per element, all kinds in one launch (Section 6.5 runs an aging
// iteration's inserts, queries and deletes concurrently in one kernel).
//
// A wave takes 64 operations at a time and runs them grouped by kind (queries,
// then inserts and upserts, then erases): tiles of a wave execute in lockstep, so
// a wave whose tiles run different kinds would go through every kind's code
// path, one after another.  Grouping leaves at most two kinds in one round of
// tiles.  The operations of a launch are concurrent, so their order within it
// is free.  Cuckoo keeps one operation per tile in input order: its three-lock
// paths need the registers the grouping takes.
//
// MERGED: the call's upserts were merged by key (hw_merge.hpp); only each key's
// leader runs its table upsert, and a follower's status is written later.  `oe`
// is the operation's op_ent word (read by the caller; unused unless MERGED).
template <class C, bool MERGED = false>
__device__ __forceinline__ void mixed_op(const TableDev& tv, const Tile<C::T>& tile, const uint8_t* __restrict__ ops,
                                         const typename C::K* __restrict__ keys,
                                         const typename C::K* __restrict__ vals, uint64_t j, int combine,
                                         typename C::K* __restrict__ out, uint8_t* __restrict__ status,
                                         const MergeWs& ws, uint32_t oe) {
  using K = typename C::K;
  const int op = ops[j];
  const K key = keys[j];
  K v = 0;
  uint8_t st;
  bool report = true;
  if (op == OP_QUERY) {
    st = Ops<C>::query(tv, tile, key, &v);
  } else if (op == OP_ERASE || op == OP_INSERT || op == OP_UPSERT) {
    const bool erase = op == OP_ERASE;
    K val = erase ? K(0) : vals[j];
    const int cmb = op == OP_UPSERT ? combine : C_KEEP;
    uint32_t e = MERGE_NONE;
    if constexpr (MERGED) {
      if (op == OP_UPSERT) {
        e = oe;
        report = merge_take<K>(ws, tile, j, oe, cmb, &val);
      }
    }
    st = ST_EXISTED;
    if (report) {
      // two call sites, each with `erase` constant: one lock loop holding both
      // critical sections measured 3-4% slower in aging launches
      st = erase ? Ops<C>::erase(tv, tile, key) : Ops<C>::upsert(tv, tile, key, val, cmb);
      if constexpr (MERGED) {
        if (e != MERGE_NONE && tile.leader()) ws.ent[e].stat = st;
      }
    }
  } else {
    st = ST_INVALID;
  }
  if (tile.leader()) {
    if (out) out[j] = v;
    if (status && report) status[j] = st;
  }
}

template <class C, bool MERGED>
__device__ __forceinline__ void mixed_body(const TableDev& tv, const uint8_t* __restrict__ ops,
                                           const typename C::K* __restrict__ keys,
                                           const typename C::K* __restrict__ vals, uint64_t n, int combine,
                                           typename C::K* __restrict__ out, uint8_t* __restrict__ status,
                                           uint8_t* order_lds, uint32_t* oent_lds, const MergeWs& ws) {
  const Tile<C::T> tile;
  if constexpr (C::CUCKOO) {
    const uint64_t stride = (uint64_t)gridDim.x * (BLOCK / C::T);
    for (uint64_t i = ((uint64_t)blockIdx.x * BLOCK + threadIdx.x) / C::T; i < n; i += stride)
      mixed_op<C, MERGED>(tv, tile, ops, keys, vals, i, combine, out, status, ws, MERGED ? ws.op_ent[i] : MERGE_NONE);
    return;
  }
  // wave-uniform values made scalar, so they take no vector registers
  const uint32_t wid = __builtin_amdgcn_readfirstlane(threadIdx.x / 64);
  uint8_t* order = order_lds + wid * 64;  // this wave's 64 entries
  uint32_t* oent = oent_lds + (MERGED ? wid * 64 : 0);
  const uint32_t lane = __lane_id();
  const uint64_t wave = (uint64_t)blockIdx.x * (BLOCK / 64) + wid;
  const uint64_t n_waves = (uint64_t)gridDim.x * (BLOCK / 64);
  for (uint64_t base = wave * 64; base < n; base += n_waves * 64) {
    // rank of the lane's operation: query 0, insert/upsert 1, erase 2, other 3,
    // nothing to do 4 (an upsert that the merge's build pass found to follow
    // another: the finishing pass reports it), past the end 5; its place =
    // lanes of lower rank + lower lanes of its rank
    const uint64_t i = base + lane;
    int r = 5;
    uint32_t oe = MERGE_NONE;
    if (i < n) {
      const int op = ops[i];
      r = op == OP_QUERY ? 0 : (op == OP_INSERT || op == OP_UPSERT) ? 1 : op == OP_ERASE ? 2 : 3;
      if constexpr (MERGED) {
        if (op == OP_UPSERT) {
          oe = ws.op_ent[i];
          if (oe != MERGE_NONE && (oe & MERGE_FOLLOWER)) {
            r = 4;
            if (out) out[i] = 0;
          }
        }
      }
    }
    uint32_t place = 0;
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      const uint64_t m = __ballot(r == k);
      if (k < r) place += (uint32_t)__popcll(m);
      if (k == r) place += (uint32_t)__popcll(m & ((1ull << lane) - 1));
    }
    if (r == 5) place = lane;  // past-end lanes are the highest ones
    order[place] = (uint8_t)lane;
    if constexpr (MERGED) oent[place] = oe;
    const uint32_t cnt = (uint32_t)__popcll(__ballot(r < 4));
    wave_sync();
    for (uint32_t s = lane / C::T; s < cnt; s += 64 / C::T)
      mixed_op<C, MERGED>(tv, tile, ops, keys, vals, base + order[s], combine, out, status, ws,
                          MERGED ? oent[s] : MERGE_NONE);
    wave_sync();  // the next window rewrites `order`
  }
}

template <class C, bool MERGED = false>
__global__ void __launch_bounds__(BLOCK)
k_mixed(TableDev tv, const uint8_t* __restrict__ ops, const typename C::K* __restrict__ keys,
        const typename C::K* __restrict__ vals, uint64_t n, int combine, typename C::K* __restrict__ out,
        uint8_t* __restrict__ status, MergeWs ws) {
  __shared__ uint8_t order_lds[BLOCK];
  __shared__ uint32_t oent_lds[MERGED ? BLOCK : 1];
  mixed_body<C, MERGED>(tv, ops, keys, vals, n, combine, out, status, order_lds, oent_lds, ws);
}

// With an occupancy bound of W waves per SIMD: the grouping's registers would
// cost iceberg its sixth wave and the double-hashing and two-choice designs
// their eighth.  A 2^20-operation launch is 16384 windows: at 8 waves/SIMD the
// chip holds 8192 waves and runs them in two rounds, at 7 it needs three.  The
// bound costs the two-choice designs 12-24 bytes of spill per lane.
template <class C, int W, bool MERGED = false>
__global__ void __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(W, 8)))
k_mixed_w(TableDev tv, const uint8_t* __restrict__ ops, const typename C::K* __restrict__ keys,
           const typename C::K* __restrict__ vals, uint64_t n, int combine, typename C::K* __restrict__ out,
           uint8_t* __restrict__ status, MergeWs ws) {
  __shared__ uint8_t order_lds[BLOCK];
  __shared__ uint32_t oent_lds[MERGED ? BLOCK : 1];
  mixed_body<C, MERGED>(tv, ops, keys, vals, n, combine, out, status, order_lds, oent_lds, ws);
}

// Host side ------------------------------------------------------------------

struct LaunchArgs {
  TableDev tv;
  unsigned max_blocks;  // grid cap (device-dependent)
};

inline unsigned grid_for(uint64_t n, int T, unsigned max_blocks) {
  const uint64_t per_block = BLOCK / T;
  uint64_t blocks = (n + per_block - 1) / per_block;
  if (blocks > max_blocks) blocks = max_blocks;
  return (unsigned)(blocks ? blocks : 1);
}

typedef hipError_t (*upsert_fn)(const LaunchArgs&, const void*, const void*, uint64_t, int, uint8_t*,
                                hipStream_t);
typedef hipError_t (*query_fn)(const LaunchArgs&, const void*, uint64_t, void*, uint8_t*, hipStream_t);
typedef hipError_t (*erase_fn)(const LaunchArgs&, const void*, uint64_t, uint8_t*, hipStream_t);
typedef hipError_t (*mixed_fn)(const LaunchArgs&, const uint8_t*, const void*, const void*, uint64_t,
                               int, void*, uint8_t*, const MergeWs*, hipStream_t);

struct KernelSet {
  int kv_bits, design, bucket, tile;
  bool bsp;  // phased variant (no locks, plain loads in queries)
  upsert_fn upsert;
  query_fn query;
  erase_fn erase;
  mixed_fn mixed;
};

template <class C>
struct Launch {
  using K = typename C::K;
  static hipError_t upsert(const LaunchArgs& a, const void* keys, const void* vals, uint64_t n,
                           int combine, uint8_t* status, hipStream_t s) {
    if (a.tv.aggregate && combine != C_REPLACE) {
      // one wave per window of AGG_WIN operations
      hipLaunchKernelGGL((k_upsert_agg<C>), dim3(grid_for((n + AGG_WIN - 1) / AGG_WIN, 64, a.max_blocks)),
                         dim3(BLOCK), 0, s, a.tv, (const K*)keys, (const K*)vals, n, combine, status);
      if (a.tv.hot_tag && combine != C_KEEP)
        hipLaunchKernelGGL((k_hot_flush<K>), dim3(HOT_N / BLOCK), dim3(BLOCK), 0, s, a.tv);
    } else {
      hipLaunchKernelGGL((k_upsert<C>), dim3(grid_for(n, C::T, a.max_blocks)), dim3(BLOCK), 0, s, a.tv,
                         (const K*)keys, (const K*)vals, n, combine, status);
    }
    return hipGetLastError();
  }
  static hipError_t query(const LaunchArgs& a, const void* keys, uint64_t n, void* out, uint8_t* found,
                          hipStream_t s) {
    hipLaunchKernelGGL((k_query<C>), dim3(grid_for(n, C::T, a.max_blocks)), dim3(BLOCK), 0, s, a.tv,
                       (const K*)keys, n, (K*)out, found);
    return hipGetLastError();
  }
  static hipError_t erase(const LaunchArgs& a, const void* keys, uint64_t n, uint8_t* found,
                          hipStream_t s) {
    hipLaunchKernelGGL((k_erase<C>), dim3(grid_for(n, C::T, a.max_blocks)), dim3(BLOCK), 0, s, a.tv,
                       (const K*)keys, n, found);
    return hipGetLastError();
  }
  // One kernel launch of the mixed kernel over ops [0, n).
  template <bool MERGED>
  static void mixed_launch(const LaunchArgs& a, const uint8_t* ops, const K* keys, const K* vals, uint64_t n,
                           int combine, K* out, uint8_t* status, const MergeWs& ws, hipStream_t s) {
    if constexpr (C::CUCKOO)
      hipLaunchKernelGGL((k_mixed<C, MERGED>), dim3(grid_for(n, C::T, a.max_blocks)), dim3(BLOCK), 0, s, a.tv, ops,
                         keys, vals, n, combine, out, status, ws);
    else if constexpr (C::ICEBERG && C::T >= 4)  // one wave per window of 64 operations
      hipLaunchKernelGGL((k_mixed_w<C, 6, MERGED>), dim3(grid_for((n + 63) / 64, 64, a.max_blocks)), dim3(BLOCK),
                         0, s, a.tv, ops, keys, vals, n, combine, out, status, ws);
    else if constexpr (!C::ICEBERG && !C::CHAIN && C::T >= 4)  // double hashing, two-choice
      hipLaunchKernelGGL((k_mixed_w<C, 8, MERGED>), dim3(grid_for((n + 63) / 64, 64, a.max_blocks)), dim3(BLOCK),
                         0, s, a.tv, ops, keys, vals, n, combine, out, status, ws);
    else
      hipLaunchKernelGGL((k_mixed<C, MERGED>), dim3(grid_for((n + 63) / 64, 64, a.max_blocks)), dim3(BLOCK), 0, s,
                         a.tv, ops, keys, vals, n, combine, out, status, ws);
  }

  // ws non-null (and a mergeable combine): the call's upserts are merged by key,
  // chunk by chunk of at most ws->chunk operations (hw_merge.hpp).  Chunks run
  // one after another, which is one serialisation of the call.
  static hipError_t mixed(const LaunchArgs& a, const uint8_t* ops, const void* keys, const void* vals,
                          uint64_t n, int combine, void* out, uint8_t* status, const MergeWs* ws, hipStream_t s) {
    const K* k = (const K*)keys;
    const K* v = (const K*)vals;
    K* o = (K*)out;
    if (!ws || combine == C_REPLACE || !vals) {
      mixed_launch<false>(a, ops, k, v, n, combine, o, status, MergeWs{}, s);
      return hipGetLastError();
    }
    for (uint64_t off = 0; off < n; off += ws->chunk) {
      const uint64_t m = n - off < ws->chunk ? n - off : ws->chunk;
      const unsigned gb = (unsigned)((m + MERGE_BLOCK_OPS - 1) / MERGE_BLOCK_OPS);
      hipLaunchKernelGGL((k_merge_build<K>), dim3(gb < a.max_blocks ? gb : a.max_blocks), dim3(MERGE_THREADS), 0, s, *ws,
                         ops + off, k + off, v + off, m, combine);
      mixed_launch<true>(a, ops + off, k + off, v + off, m, combine, o ? o + off : nullptr,
                         status ? status + off : nullptr, *ws, s);
      hipLaunchKernelGGL((k_merge_finish<K>), dim3(grid_for(m, 1, a.max_blocks)), dim3(256), 0, s, *ws, ops + off, m,
                         status ? status + off : nullptr);
      const hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
    return hipGetLastError();
  }
};

template <class C>
constexpr KernelSet make_set() {
  return KernelSet{(int)sizeof(typename C::K) * 8, C::DESIGN, C::B, C::T, C::BSP, &Launch<C>::upsert,
                   &Launch<C>::query, &Launch<C>::erase, &Launch<C>::mixed};
}

// Instance tables, one per translation unit.
const KernelSet* sets_u64_double(size_t* n);
const KernelSet* sets_u64_p2(size_t* n);
const KernelSet* sets_u32_double(size_t* n);
const KernelSet* sets_u32_p2(size_t* n);
const KernelSet* sets_u64_iceberg(size_t* n);
const KernelSet* sets_u32_iceberg(size_t* n);
const KernelSet* sets_u64_bsp(size_t* n);
const KernelSet* sets_u64_chain(size_t* n);
const KernelSet* sets_u64_cuckoo(size_t* n);

}  // namespace hw
