// Instantiates the kernels for dim = 2, polydeg = 6.
#include "registry.h"

namespace dgx {
const Launchers* launchers_d2_n6() {
  static const Launchers L = Launch<2, 6>::make();
  return &L;
}
}  // namespace dgx
