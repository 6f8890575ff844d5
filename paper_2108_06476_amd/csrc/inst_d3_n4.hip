// Instantiates the kernels for dim = 3, polydeg = 4.
#include "registry.h"

namespace dgx {
const Launchers* launchers_d3_n4() {
  static const Launchers L = Launch<3, 4>::make();
  return &L;
}
}  // namespace dgx
