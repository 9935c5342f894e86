// Instantiations of the advection kernels: 2D orders {0, 1, 2, 3, 4, 5}, 3D orders {0, 1, 2, 3, 4}.
#include "registry.hpp"

namespace adg {

const Launchers* find_advection(int dim, int order, int prec, bool st) {
  if (dim == 2) return pick_order<Advection, 2, 0, 1, 2, 3, 4, 5>(order, prec, st);
  if (dim == 3) return pick_order<Advection, 3, 0, 1, 2, 3, 4>(order, prec, st);
  return nullptr;
}

}  // namespace adg
