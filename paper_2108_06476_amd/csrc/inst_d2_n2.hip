// Instantiates the kernels for dim = 2, polydeg = 2.
#include "registry.h"

namespace dgx {
const Launchers* launchers_d2_n2() {
  static const Launchers L = Launch<2, 2>::make();
  return &L;
}
}  // namespace dgx
