// Instantiations of the elastic kernels: 2D orders {1, 2, 3, 4}, 3D orders {1, 2, 3, 4, 5}.
#include "registry.hpp"

namespace adg {

const Launchers* find_elastic(int dim, int order, int prec, bool st) {
  if (dim == 2) return pick_order<Elastic, 2, 1, 2, 3, 4>(order, prec, st);
  if (dim == 3) return pick_order<Elastic, 3, 1, 2, 3, 4, 5>(order, prec, st);
  return nullptr;
}

}  // namespace adg
