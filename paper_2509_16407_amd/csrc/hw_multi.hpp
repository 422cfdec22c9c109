// One persistent launch serving many tables of uneven capacities and configurations.
//
// Work is a list of items (table, operation kind, op range [begin, end)) over shared
// key / value / output arrays.  Items are spread over NQ queues, each a slice of the
// item array with its own head counter, so popping never funnels through a single
// atomic address.  A wave starts at its home queue (block index mod NQ: workgroups
// are dealt to the XCDs round-robin, so items of small tables, which the host puts
// on queue table mod NQ, stay near one XCD's L2) and then takes work from the other
// queues until every queue is empty; each wave visits each queue at most once after
// finding it empty, so every wave exits.
//
// Per item, a wave-uniform switch selects the table's compiled configuration from a
// menu and runs the same per-operation code as the single-table kernels, with the
// wave's 64 lanes split into tiles of that configuration's width.
#pragma once

#include "hw_launch.hpp"

namespace hw {

constexpr int NQ = 8;
// Queue head counters sit one per 128-byte line (HEAD_STRIDE 32-bit words
// apart): atomics to one line are served one after another.
constexpr int HEAD_STRIDE = 32;

#ifndef HW_MULTI_WAVES
#define HW_MULTI_WAVES 6  // occupancy target of the multi-table kernel (waves per SIMD)
#endif
#ifndef HW_SOLO_WAVES
#define HW_SOLO_WAVES 8   // occupancy target of its single-configuration instances
#endif
#ifndef HW_SOLO_AGG_WAVES
#define HW_SOLO_AGG_WAVES 6  // the same with the merging path compiled in (~80 VGPRs)
#endif

struct MultiItem {
  uint32_t table;
  uint32_t op;     // low byte: OP_*; bits 8..15: combine for OP_UPSERT
  uint64_t begin;  // ops [begin, end) of the shared arrays
  uint64_t end;
};

struct MultiTable {
  TableDev tv;
  uint32_t cls;          // index in the key width's configuration menu
  uint32_t pad;
  uint64_t fill_words;   // 16-byte words of slots + tags (all-ones when empty)
  uint64_t zero_words;   // 16-byte words of locks + control (zero when empty)
};

struct MultiQueues {
  uint32_t start[NQ];  // item index where queue q starts
  uint32_t end[NQ];
};

template <bool AGG, class C0, class... Cs>
struct Menu {
  static constexpr int N = 1 + sizeof...(Cs);
  static constexpr bool AGGREGATE = AGG;  // compiled with the merging path (hw_agg.hpp)
  using K = typename C0::K;               // one key width per menu
  // occupancy target: cuckoo's three-lock paths need more registers
  static constexpr int WAVES = (C0::CUCKOO || ... || Cs::CUCKOO) ? 4 : HW_MULTI_WAVES;
};

// A menu of one configuration with its own occupancy target.  A group whose
// tables all share one configuration runs on it: the switch over the menu and
// the other configurations' inlined paths cost the full menu's kernel registers
// and spills, and with them two of its eight waves per SIMD.
template <class M, int W>
struct Solo : M {
  static constexpr int WAVES = W;
};

// Occupancy target of configuration C's own kernel, with or without the merging
// path compiled in.
template <class C>
constexpr int solo_waves(bool agg) {
  return C::CUCKOO ? 4 : C::ICEBERG ? 6 : agg ? HW_SOLO_AGG_WAVES : HW_SOLO_WAVES;
}

// Runs ops [m.begin, m.end) of one table with configuration C on this wave.
template <class C, bool AGG>
__device__ __forceinline__ void run_item(const TableDev& tv, const MultiItem& m, const typename C::K* __restrict__ keys,
                         const typename C::K* __restrict__ vals, typename C::K* __restrict__ out,
                         uint8_t* __restrict__ status, AggLds<typename C::K>& agg) {
  using K = typename C::K;
  const Tile<C::T> tile;
  const uint32_t lane = __lane_id();
  const int op = (int)(m.op & 0xFF);
  const int combine = op == OP_INSERT ? C_KEEP : (int)((m.op >> 8) & 0xFF);
  if constexpr (AGG) {
    if ((op == OP_INSERT || op == OP_UPSERT) && tv.aggregate && agg_merges(combine)) {
      for (uint64_t i0 = m.begin; i0 < m.end; i0 += AGG_WIN) {
        const uint64_t left = m.end - i0;
        agg_window<C>(tv, agg, keys, vals, i0, (uint32_t)(left < AGG_WIN ? left : AGG_WIN), combine, status,
                      (blockIdx.x * (BLOCK / 64) + threadIdx.x / 64) % HOT_ROWS);
      }
      return;
    }
  }
  for (uint64_t i = m.begin + lane / C::T; i < m.end; i += 64 / C::T) {
    const K key = keys[i];
    uint8_t st;
    if (op == OP_QUERY) {
      K v;
      st = Ops<C>::query(tv, tile, key, &v);
      if (out && tile.leader()) out[i] = v;
    } else if (op == OP_ERASE) {
      st = Ops<C>::erase(tv, tile, key);
    } else {
      st = Ops<C>::upsert(tv, tile, key, vals[i], combine);
    }
    if (status && tile.leader()) status[i] = st;
  }
}

template <bool AGG, class... Cs>
__device__ __forceinline__ void dispatch(uint32_t cls, const TableDev& tv, const MultiItem& m,
                                         const void* keys, const void* vals, void* out, uint8_t* status,
                                         AggLds<typename Menu<AGG, Cs...>::K>& agg, Menu<AGG, Cs...>) {
  uint32_t i = 0;
  (void)((cls == i++ ? (run_item<Cs, AGG>(tv, m, (const typename Cs::K*)keys, (const typename Cs::K*)vals,
                                     (typename Cs::K*)out, status, agg),
                        true)
                     : false) ||
         ...);
}

template <class M>
__global__ void __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(M::WAVES, 8)))
k_multi(const MultiTable* __restrict__ tables, const MultiItem* __restrict__ items, MultiQueues qs,
        uint32_t* heads, const void* keys, const void* vals, void* out, uint8_t* status) {
  __shared__ AggLds<typename M::K> agg_lds[M::AGGREGATE ? BLOCK / 64 : 1];
  AggLds<typename M::K>& agg = agg_lds[M::AGGREGATE ? threadIdx.x / 64 : 0];
  const uint32_t lane = __lane_id();
  const uint32_t home = blockIdx.x % NQ;
  for (uint32_t k = 0; k < NQ; ++k) {
    const uint32_t q = (home + k) % NQ;
    const uint32_t qlen = qs.end[q] - qs.start[q];
    while (true) {
      uint32_t idx = 0;
      if (lane == 0)
        idx = __hip_atomic_fetch_add(heads + q * HEAD_STRIDE, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      idx = __builtin_amdgcn_readfirstlane(idx);
      if (idx >= qlen) break;
      const MultiItem m = items[qs.start[q] + idx];
      const MultiTable& t = tables[m.table];
      dispatch(__builtin_amdgcn_readfirstlane(t.cls), t.tv, m, keys, vals, out, status, agg, M{});
    }
  }
}

// Configuration menus of the multi-table kernel (one per key width).  The
// autotuner chooses among these.
// The 64-bit menu carries the merging path (hw_agg.hpp) for tables created with
// HWAVE_F_AGGREGATE; the 32-bit menu does not (its register budget is tighter).
using MenuU64 = Menu<true, Cfg<uint64_t, D_DOUBLE, 8, 8>, Cfg<uint64_t, D_DOUBLE, 16, 8>,
                     Cfg<uint64_t, D_DOUBLE_M, 32, 4>, Cfg<uint64_t, D_DOUBLE_M, 32, 8>,
                     Cfg<uint64_t, D_P2, 32, 8>, Cfg<uint64_t, D_P2_M, 32, 4>,
                     Cfg<uint64_t, D_P2_M, 32, 8>, Cfg<uint64_t, D_P2_M, 64, 8>>;
// Extended 64-bit menu: the base menu plus iceberg, chaining and cuckoo.  A
// group that holds a table of these designs runs on it; its inlined paths cost
// registers (and spills), so groups of base designs keep the base menu.
using MenuU64X = Menu<true, Cfg<uint64_t, D_DOUBLE, 8, 8>, Cfg<uint64_t, D_DOUBLE, 16, 8>,
                      Cfg<uint64_t, D_DOUBLE_M, 32, 4>, Cfg<uint64_t, D_DOUBLE_M, 32, 8>,
                      Cfg<uint64_t, D_P2, 32, 8>, Cfg<uint64_t, D_P2_M, 32, 4>,
                      Cfg<uint64_t, D_P2_M, 32, 8>, Cfg<uint64_t, D_P2_M, 64, 8>,
                      Cfg<uint64_t, D_ICEBERG, 32, 8>, Cfg<uint64_t, D_ICEBERG_M, 32, 4>,
                      Cfg<uint64_t, D_CHAINING, 7, 8>, Cfg<uint64_t, D_CUCKOO, 8, 4>>;
using MenuU32 = Menu<false, Cfg<uint32_t, D_DOUBLE, 16, 4>, Cfg<uint32_t, D_DOUBLE, 16, 8>,
                     Cfg<uint32_t, D_DOUBLE, 32, 16>, Cfg<uint32_t, D_DOUBLE, 64, 32>,
                     Cfg<uint32_t, D_DOUBLE, 128, 64>, Cfg<uint32_t, D_DOUBLE_M, 32, 4>,
                     Cfg<uint32_t, D_P2, 32, 8>, Cfg<uint32_t, D_P2_M, 16, 4>,
                     Cfg<uint32_t, D_P2_M, 32, 4>, Cfg<uint32_t, D_P2_M, 32, 8>>;

struct MenuEntry {
  int design, bucket, tile;
};

template <bool AGG, class... Cs>
inline const MenuEntry* menu_entries(Menu<AGG, Cs...>, int* n) {
  static const MenuEntry e[] = {MenuEntry{Cs::DESIGN, Cs::B, Cs::T}...};
  *n = (int)sizeof...(Cs);
  return e;
}

// Host launchers (inst_multi.hip).
hipError_t launch_multi_clear(unsigned grid, const MultiTable* tables, uint32_t n_tables, hipStream_t s);
// menu: MENU_BASE, MENU_EXT (64-bit keys only) or MENU_SOLO, the one-entry menu
// of entry `solo` of the 32-bit menu or of the 64-bit extended menu (whose first
// entries are the base menu's); every table's `cls` is then 0.  `agg`: a 64-bit
// solo kernel with the merging path (some table of the group merges duplicates).
enum : int { MENU_BASE = 0, MENU_EXT = 1, MENU_SOLO = 2 };
hipError_t launch_multi(int kv_bits, int menu, int solo, bool agg, unsigned grid, const MultiTable* tables,
                        const MultiItem* items, const MultiQueues& qs, uint32_t* heads, const void* keys,
                        const void* vals, void* out, uint8_t* status, hipStream_t s);
// Single-configuration instances (inst_multi_solo.hip): entry `solo` of the
// 32-bit menu or the 64-bit extended menu, with or without the merging path
// (64-bit keys only), and their occupancy targets.
int multi_solo_waves(int kv_bits, int solo, bool agg);
hipError_t launch_multi_solo(int kv_bits, int solo, bool agg, unsigned grid, const MultiTable* tables,
                             const MultiItem* items, const MultiQueues& qs, uint32_t* heads, const void* keys,
                             const void* vals, void* out, uint8_t* status, hipStream_t s);
// Occupancy target (waves per SIMD) of a menu's kernel, for the persistent grid.
int multi_waves(int kv_bits, int menu, int solo, bool agg);
// Folds the hot-key accumulators of the n_hot tables listed in `hot` (device
// array of table indices); a no-op for n_hot == 0.
hipError_t launch_multi_hot_flush(int kv_bits, const MultiTable* tables, const uint32_t* hot, uint32_t n_hot,
                                  hipStream_t s);
int multi_menu_index(int kv_bits, int menu, int design, int bucket, int tile);

}  // namespace hw
