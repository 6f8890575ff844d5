// Instantiates the kernels for dim = 2, polydeg = 7.
#include "registry.h"

namespace dgx {
const Launchers* launchers_d2_n7() {
  static const Launchers L = Launch<2, 7>::make();
  return &L;
}
}  // namespace dgx
