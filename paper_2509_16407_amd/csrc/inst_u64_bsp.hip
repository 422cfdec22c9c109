// Kernel instances of the phased (bulk-synchronous) variant: 64-bit keys/values,
// every design at its default configuration (Section 5).  Used to measure what
// full concurrency costs (Section 6.4, Table 1's phased query column).  Chaining
// and cuckoo keep their write locks; their queries take none.
#include "hw_launch.hpp"

namespace hw {
const KernelSet* sets_u64_bsp(size_t* n) {
  static const KernelSet s[] = {
      make_set<Cfg<uint64_t, D_DOUBLE, 8, 8, true>>(),     make_set<Cfg<uint64_t, D_DOUBLE_M, 32, 4, true>>(),
      make_set<Cfg<uint64_t, D_P2, 32, 8, true>>(),        make_set<Cfg<uint64_t, D_P2_M, 32, 4, true>>(),
      make_set<Cfg<uint64_t, D_ICEBERG, 32, 8, true>>(),   make_set<Cfg<uint64_t, D_ICEBERG_M, 32, 4, true>>(),
      make_set<Cfg<uint64_t, D_CHAINING, 7, 8, true>>(),   make_set<Cfg<uint64_t, D_CUCKOO, 8, 4, true>>(),
  };
  *n = sizeof(s) / sizeof(s[0]);
  return s;
}
}  // namespace hw
