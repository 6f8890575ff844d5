// Instantiates the kernels for dim = 3, polydeg = 7.
#include "registry.h"

namespace dgx {
const Launchers* launchers_d3_n7() {
  static const Launchers L = Launch<3, 7>::make();
  return &L;
}
}  // namespace dgx
