// Instantiates the kernels for dim = 3, polydeg = 2.
#include "registry.h"

namespace dgx {
const Launchers* launchers_d3_n2() {
  static const Launchers L = Launch<3, 2>::make();
  return &L;
}
}  // namespace dgx
