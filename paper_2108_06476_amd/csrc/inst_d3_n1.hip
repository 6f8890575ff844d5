// Instantiates the kernels for dim = 3, polydeg = 1.
#include "registry.h"

namespace dgx {
const Launchers* launchers_d3_n1() {
  static const Launchers L = Launch<3, 1>::make();
  return &L;
}
}  // namespace dgx
