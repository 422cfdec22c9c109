// Single-configuration instances of the multi-table kernel: one per entry of
// the 32-bit menu and of the 64-bit extended menu (the base menu's entries come
// first in it), the 64-bit ones with and without the merging path.
#include "hw_multi.hpp"

namespace hw {

namespace {

template <class C, bool AGG>
void launch_one(unsigned grid, const MultiTable* tables, const MultiItem* items, const MultiQueues& qs,
                uint32_t* heads, const void* keys, const void* vals, void* out, uint8_t* status, hipStream_t s) {
  hipLaunchKernelGGL((k_multi<Solo<Menu<AGG, C>, solo_waves<C>(AGG)>>), dim3(grid), dim3(BLOCK), 0, s, tables,
                     items, qs, heads, keys, vals, out, status);
}

// Launches entry `solo` of the menu, compiled with merging path AGG; false if
// there is no such entry.
template <bool AGG, bool MENU_AGG, class... Cs>
bool launch_entry(Menu<MENU_AGG, Cs...>, int solo, unsigned grid, const MultiTable* tables, const MultiItem* items,
                  const MultiQueues& qs, uint32_t* heads, const void* keys, const void* vals, void* out,
                  uint8_t* status, hipStream_t s) {
  int i = 0;
  return ((solo == i++ ? (launch_one<Cs, AGG>(grid, tables, items, qs, heads, keys, vals, out, status, s), true)
                       : false) ||
          ...);
}

template <bool MENU_AGG, class... Cs>
int waves_of_entry(Menu<MENU_AGG, Cs...>, int solo, bool agg) {
  int i = 0, w = 0;
  (void)((solo == i++ ? (w = solo_waves<Cs>(agg), true) : false) || ...);
  return w;
}

}  // namespace

int multi_solo_waves(int kv_bits, int solo, bool agg) {
  return kv_bits == 64 ? waves_of_entry(MenuU64X{}, solo, agg) : waves_of_entry(MenuU32{}, solo, false);
}

hipError_t launch_multi_solo(int kv_bits, int solo, bool agg, unsigned grid, const MultiTable* tables,
                             const MultiItem* items, const MultiQueues& qs, uint32_t* heads, const void* keys,
                             const void* vals, void* out, uint8_t* status, hipStream_t s) {
  bool ok;
  if (kv_bits == 64 && agg)
    ok = launch_entry<true>(MenuU64X{}, solo, grid, tables, items, qs, heads, keys, vals, out, status, s);
  else if (kv_bits == 64)
    ok = launch_entry<false>(MenuU64X{}, solo, grid, tables, items, qs, heads, keys, vals, out, status, s);
  else
    ok = launch_entry<false>(MenuU32{}, solo, grid, tables, items, qs, heads, keys, vals, out, status, s);
  return ok ? hipGetLastError() : hipErrorInvalidValue;
}

}  // namespace hw
