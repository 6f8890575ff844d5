// Instantiates the kernels for dim = 2, polydeg = 5.
#include "registry.h"

namespace dgx {
const Launchers* launchers_d2_n5() {
  static const Launchers L = Launch<2, 5>::make();
  return &L;
}
}  // namespace dgx
