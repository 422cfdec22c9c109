// Single-configuration instances of the multi-table kernel: one per entry of
// each key width's base menu; 64-bit entries also without the merging path.
#include "hw_multi.hpp"

namespace hw {

namespace {

template <class C, bool AGG>
void launch_one(unsigned grid, const MultiTable* tables, const MultiItem* items, const MultiQueues& qs,
                uint32_t* heads, const void* keys, const void* vals, void* out, uint8_t* status, hipStream_t s) {
  hipLaunchKernelGGL((k_multi<Solo<Menu<AGG, C>, AGG ? HW_SOLO_AGG_WAVES : HW_SOLO_WAVES>>), dim3(grid),
                     dim3(BLOCK), 0, s, tables, items, qs, heads, keys, vals, out, status);
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

}  // namespace

hipError_t launch_multi_solo(int kv_bits, int solo, bool agg, unsigned grid, const MultiTable* tables,
                             const MultiItem* items, const MultiQueues& qs, uint32_t* heads, const void* keys,
                             const void* vals, void* out, uint8_t* status, hipStream_t s) {
  bool ok;
  if (kv_bits == 64 && agg)
    ok = launch_entry<true>(MenuU64{}, solo, grid, tables, items, qs, heads, keys, vals, out, status, s);
  else if (kv_bits == 64)
    ok = launch_entry<false>(MenuU64{}, solo, grid, tables, items, qs, heads, keys, vals, out, status, s);
  else
    ok = launch_entry<false>(MenuU32{}, solo, grid, tables, items, qs, heads, keys, vals, out, status, s);
  return ok ? hipGetLastError() : hipErrorInvalidValue;
}

}  // namespace hw
