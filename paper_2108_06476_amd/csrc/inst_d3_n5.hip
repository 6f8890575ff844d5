// Instantiates the kernels for dim = 3, polydeg = 5.
#include "registry.h"

namespace dgx {
const Launchers* launchers_d3_n5() {
  static const Launchers L = Launch<3, 5>::make();
  return &L;
}
}  // namespace dgx
