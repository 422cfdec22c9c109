// Kernel instances: 64-bit keys/values, three-way bucketed cuckoo hashing
// (Section 5: buckets of 8 pairs in one cache line, 4 lanes per tile).
#include "hw_launch.hpp"

namespace hw {
const KernelSet* sets_u64_cuckoo(size_t* n) {
  static const KernelSet s[] = {
      make_set<Cfg<uint64_t, D_CUCKOO, 8, 4>>(),
      make_set<Cfg<uint64_t, D_CUCKOO, 8, 8>>(),
      make_set<Cfg<uint64_t, D_CUCKOO, 16, 8>>(),
  };
  *n = sizeof(s) / sizeof(s[0]);
  return s;
}
}  // namespace hw
