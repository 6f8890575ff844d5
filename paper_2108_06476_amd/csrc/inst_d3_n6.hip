// Instantiates the kernels for dim = 3, polydeg = 6.
#include "registry.h"

namespace dgx {
const Launchers* launchers_d3_n6() {
  static const Launchers L = Launch<3, 6>::make();
  return &L;
}
}  // namespace dgx
