// Kernel instances: 64-bit keys/values, power-of-two-choice (with and without tags).
#include "hw_launch.hpp"

namespace hw {
const KernelSet* sets_u64_p2(size_t* n) {
  static const KernelSet s[] = {
      make_set<Cfg<uint64_t, D_P2, 16, 8>>(),   make_set<Cfg<uint64_t, D_P2, 32, 4>>(),
      make_set<Cfg<uint64_t, D_P2, 32, 8>>(),   make_set<Cfg<uint64_t, D_P2, 32, 16>>(),
      make_set<Cfg<uint64_t, D_P2, 32, 32>>(),  make_set<Cfg<uint64_t, D_P2_M, 16, 4>>(),   make_set<Cfg<uint64_t, D_P2_M, 32, 2>>(),
      make_set<Cfg<uint64_t, D_P2_M, 32, 4>>(), make_set<Cfg<uint64_t, D_P2_M, 32, 8>>(),
      make_set<Cfg<uint64_t, D_P2_M, 32, 16>>(), make_set<Cfg<uint64_t, D_P2_M, 64, 8>>(),
  };
  *n = sizeof(s) / sizeof(s[0]);
  return s;
}
}  // namespace hw
