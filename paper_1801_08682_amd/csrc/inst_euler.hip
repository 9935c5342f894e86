// Instantiations of the euler kernels: 2D orders {0, 1, 2, 3, 4, 5}, 3D orders {0, 1, 2, 3, 4, 5, 7}.
#include "registry.hpp"

namespace adg {

const Launchers* find_euler(int dim, int order, int prec, bool st) {
  if (dim == 2) return pick_order<Euler, 2, 0, 1, 2, 3, 4, 5>(order, prec, st);
  if (dim == 3) return pick_order<Euler, 3, 0, 1, 2, 3, 4, 5, 7>(order, prec, st);
  return nullptr;
}

}  // namespace adg
