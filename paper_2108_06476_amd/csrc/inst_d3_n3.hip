// Instantiates the kernels for dim = 3, polydeg = 3.
#include "registry.h"

namespace dgx {
const Launchers* launchers_d3_n3() {
  static const Launchers L = Launch<3, 3>::make();
  return &L;
}
}  // namespace dgx
