// Instantiates the kernels for dim = 2, polydeg = 1.
#include "registry.h"

namespace dgx {
const Launchers* launchers_d2_n1() {
  static const Launchers L = Launch<2, 1>::make();
  return &L;
}
}  // namespace dgx
