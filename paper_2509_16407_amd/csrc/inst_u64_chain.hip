// Kernel instances: 64-bit keys/values, chaining (one 128-byte node of 7 pairs
// and a link per line, one lane per 16 bytes; Section 5).
#include "hw_launch.hpp"

namespace hw {
const KernelSet* sets_u64_chain(size_t* n) {
  static const KernelSet s[] = {
      make_set<Cfg<uint64_t, D_CHAINING, 7, 8>>(),
  };
  *n = sizeof(s) / sizeof(s[0]);
  return s;
}
}  // namespace hw
