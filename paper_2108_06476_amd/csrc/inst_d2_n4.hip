// Instantiates the kernels for dim = 2, polydeg = 4.
#include "registry.h"

namespace dgx {
const Launchers* launchers_d2_n4() {
  static const Launchers L = Launch<2, 4>::make();
  return &L;
}
}  // namespace dgx
