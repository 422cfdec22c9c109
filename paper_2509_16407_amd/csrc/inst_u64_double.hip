// Kernel instances: 64-bit keys/values, double hashing (with and without tags).
#include "hw_launch.hpp"

namespace hw {
const KernelSet* sets_u64_double(size_t* n) {
  static const KernelSet s[] = {
      make_set<Cfg<uint64_t, D_DOUBLE, 8, 4>>(),    make_set<Cfg<uint64_t, D_DOUBLE, 8, 8>>(),
      make_set<Cfg<uint64_t, D_DOUBLE, 16, 4>>(),   make_set<Cfg<uint64_t, D_DOUBLE, 16, 8>>(),
      make_set<Cfg<uint64_t, D_DOUBLE, 16, 16>>(),  make_set<Cfg<uint64_t, D_DOUBLE, 32, 8>>(),
      make_set<Cfg<uint64_t, D_DOUBLE, 32, 16>>(),  make_set<Cfg<uint64_t, D_DOUBLE, 32, 32>>(),
      make_set<Cfg<uint64_t, D_DOUBLE_M, 16, 4>>(), make_set<Cfg<uint64_t, D_DOUBLE_M, 32, 4>>(),
      make_set<Cfg<uint64_t, D_DOUBLE_M, 32, 8>>(), make_set<Cfg<uint64_t, D_DOUBLE_M, 32, 16>>(),
      make_set<Cfg<uint64_t, D_DOUBLE_M, 64, 8>>(), make_set<Cfg<uint64_t, D_DOUBLE_M, 32, 2>>(),
  };
  *n = sizeof(s) / sizeof(s[0]);
  return s;
}
}  // namespace hw
