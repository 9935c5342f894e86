// Instantiations of the euler kernels: 2D orders {0, 1, 2, 3, 4, 5}, 3D orders {0, 1, 2, 3, 4, 5, 7}.
#include "registry.hpp"

namespace adg {

const Launchers* find_euler(int dim, int order, int prec) {
  if (dim == 2) return pick_order<Euler, 2, 0, 1, 2, 3, 4, 5>(order, prec);
  if (dim == 3) return pick_order<Euler, 3, 0, 1, 2, 3, 4, 5, 7>(order, prec);
  return nullptr;
}

}  // namespace adg
