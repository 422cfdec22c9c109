// Kernel instances: 32-bit keys/values, iceberg hashing (with and without tags).
#include "hw_launch.hpp"

namespace hw {
const KernelSet* sets_u32_iceberg(size_t* n) {
  static const KernelSet s[] = {
      make_set<Cfg<uint32_t, D_ICEBERG, 32, 4>>(),    make_set<Cfg<uint32_t, D_ICEBERG, 32, 8>>(),
      make_set<Cfg<uint32_t, D_ICEBERG_M, 32, 4>>(),  make_set<Cfg<uint32_t, D_ICEBERG_M, 32, 8>>(),
  };
  *n = sizeof(s) / sizeof(s[0]);
  return s;
}
}  // namespace hw
