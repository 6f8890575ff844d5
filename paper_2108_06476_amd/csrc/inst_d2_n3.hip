// Instantiates the kernels for dim = 2, polydeg = 3.
#include "registry.h"

namespace dgx {
const Launchers* launchers_d2_n3() {
  static const Launchers L = Launch<2, 3>::make();
  return &L;
}
}  // namespace dgx
