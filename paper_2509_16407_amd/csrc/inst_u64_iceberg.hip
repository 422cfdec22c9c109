// Kernel instances: 64-bit keys/values, iceberg hashing (with and without tags).
#include "hw_launch.hpp"

namespace hw {
const KernelSet* sets_u64_iceberg(size_t* n) {
  static const KernelSet s[] = {
      make_set<Cfg<uint64_t, D_ICEBERG, 32, 4>>(),    make_set<Cfg<uint64_t, D_ICEBERG, 32, 8>>(),
      make_set<Cfg<uint64_t, D_ICEBERG, 32, 16>>(),   make_set<Cfg<uint64_t, D_ICEBERG_M, 32, 4>>(),  make_set<Cfg<uint64_t, D_ICEBERG_M, 32, 2>>(),
      make_set<Cfg<uint64_t, D_ICEBERG_M, 32, 8>>(),  make_set<Cfg<uint64_t, D_ICEBERG_M, 64, 8>>(),
  };
  *n = sizeof(s) / sizeof(s[0]);
  return s;
}
}  // namespace hw
