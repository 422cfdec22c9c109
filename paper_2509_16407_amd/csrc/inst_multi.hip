// Multi-table persistent kernel instances (one per key width) and menu lookup.
#include "hw_multi.hpp"

namespace hw {

__global__ void k_zero_heads(uint32_t* heads) {
  if (threadIdx.x < NQ) heads[threadIdx.x * HEAD_STRIDE] = 0;
}

hipError_t launch_multi(int kv_bits, int menu, int solo, bool agg, unsigned grid, const MultiTable* tables,
                        const MultiItem* items, const MultiQueues& qs, uint32_t* heads, const void* keys,
                        const void* vals, void* out, uint8_t* status, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_heads, dim3(1), dim3(64), 0, s, heads);
  if (menu == MENU_SOLO)
    return launch_multi_solo(kv_bits, solo, agg, grid, tables, items, qs, heads, keys, vals, out, status, s);
  if (kv_bits == 64 && menu == MENU_EXT)
    hipLaunchKernelGGL((k_multi<MenuU64X>), dim3(grid), dim3(BLOCK), 0, s, tables, items, qs, heads, keys, vals,
                       out, status);
  else if (kv_bits == 64)
    hipLaunchKernelGGL((k_multi<MenuU64>), dim3(grid), dim3(BLOCK), 0, s, tables, items, qs, heads, keys, vals,
                       out, status);
  else
    hipLaunchKernelGGL((k_multi<MenuU32>), dim3(grid), dim3(BLOCK), 0, s, tables, items, qs, heads, keys, vals,
                       out, status);
  return hipGetLastError();
}

// Folds the hot-key accumulators of tables hot[0 .. gridDim.y) (hw_launch.hpp).
template <typename K>
__global__ void __launch_bounds__(BLOCK)
k_multi_hot_flush(const MultiTable* __restrict__ tables, const uint32_t* __restrict__ hot) {
  const uint32_t i = blockIdx.x * BLOCK + threadIdx.x;
  if (i < HOT_N) hot_flush_entry<K>(tables[hot[blockIdx.y]].tv, i);
}

hipError_t launch_multi_hot_flush(int kv_bits, const MultiTable* tables, const uint32_t* hot, uint32_t n_hot,
                                  hipStream_t s) {
  if (n_hot == 0) return hipSuccess;
  if (kv_bits == 64)
    hipLaunchKernelGGL(k_multi_hot_flush<uint64_t>, dim3(HOT_N / BLOCK, n_hot), dim3(BLOCK), 0, s, tables, hot);
  else
    hipLaunchKernelGGL(k_multi_hot_flush<uint32_t>, dim3(HOT_N / BLOCK, n_hot), dim3(BLOCK), 0, s, tables, hot);
  return hipGetLastError();
}

// Empties every table of a group: one block per table at a time (grid-stride
// over tables), 16-byte stores.  Slots and tags are contiguous from `slots`, and
// locks and control are contiguous from `locks` (the table layout).
__global__ void k_multi_clear(const MultiTable* __restrict__ tables, uint32_t n_tables) {
  for (uint32_t t = blockIdx.x; t < n_tables; t += gridDim.x) {
    const MultiTable& m = tables[t];
    uint4* a = (uint4*)m.tv.slots;
    const uint4 ones = make_uint4(~0u, ~0u, ~0u, ~0u);
    for (uint64_t i = threadIdx.x; i < m.fill_words; i += blockDim.x) a[i] = ones;
    uint4* z = (uint4*)m.tv.locks.words;
    const uint4 zero = make_uint4(0, 0, 0, 0);
    for (uint64_t i = threadIdx.x; i < m.zero_words; i += blockDim.x) z[i] = zero;
  }
}

hipError_t launch_multi_clear(unsigned grid, const MultiTable* tables, uint32_t n_tables, hipStream_t s) {
  hipLaunchKernelGGL(k_multi_clear, dim3(grid), dim3(BLOCK), 0, s, tables, n_tables);
  return hipGetLastError();
}

int multi_waves(int kv_bits, int menu, int solo, bool agg) {
  if (menu == MENU_SOLO) return multi_solo_waves(kv_bits, solo, agg);
  if (kv_bits == 64 && menu == MENU_EXT) return MenuU64X::WAVES;
  return kv_bits == 64 ? MenuU64::WAVES : MenuU32::WAVES;
}

int multi_menu_index(int kv_bits, int menu, int design, int bucket, int tile) {
  int n = 0;
  if (kv_bits != 64 && menu == MENU_EXT) return -1;
  if (menu == MENU_SOLO) menu = kv_bits == 64 ? MENU_EXT : MENU_BASE;
  const MenuEntry* e = kv_bits != 64        ? menu_entries(MenuU32{}, &n)
                       : menu == MENU_EXT ? menu_entries(MenuU64X{}, &n)
                                          : menu_entries(MenuU64{}, &n);
  for (int i = 0; i < n; i++)
    if (e[i].design == design && e[i].bucket == bucket && e[i].tile == tile) return i;
  return -1;
}

}  // namespace hw
