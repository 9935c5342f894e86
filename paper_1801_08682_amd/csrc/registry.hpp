// Compile-time registry: which (dim, order, precision, trace kind)
// combinations of a PDE are instantiated.  Included by exactly one instantiation unit per PDE.
#pragma once

#include "kernels_adj.hpp"
#include "kernels_fv.hpp"

namespace adg {

// The bfloat16 predictor (matrix-core contractions) is compiled for the
// benchmark workloads' orders and the small orders of the tests: 3D Euler
// N = 3, 4, 7, 3D elasticity N = 5, 3D acoustics N = 3.
template <template <int> class PDET, int D, int N>
constexpr bool bf16_instantiated() {
  if constexpr (D != 3) return false;
  else if constexpr (std::is_same<PDET<3>, Euler<3>>::value) return N == 3 || N == 4 || N == 7;
  else if constexpr (std::is_same<PDET<3>, Elastic<3>>::value) return N == 5;
  else if constexpr (std::is_same<PDET<3>, Acoustic<3>>::value) return N == 3;
  else return false;
}

template <template <int> class PDET, int D, int N>
const Launchers* pick_precision(int prec, bool st) {
  if (st) {     // space-time traces: float64 or float predictor (not the matrix-core one)
    if (prec == 0) {
      static const Launchers L = make_fwd_launchers<Fwd<D, N, PDET, double, true>>();
      return &L;
    }
    if (prec == 1) {
      static const Launchers L = make_fwd_launchers<Fwd<D, N, PDET, float, true>>();
      return &L;
    }
    return nullptr;
  }
  if (prec == 0) {
    using K = Fwd<D, N, PDET, double>;
    static const Launchers L = [] {
      Launchers l = make_fwd_launchers<K>();
      l.adjoint = &launch_adjoint<K>;
      l.fv_project = &launch_fv_project<K>;
      l.fv_reconstruct = &launch_fv_reconstruct<K>;
      l.fv_step = &launch_fv_step<K>;
      l.adj_slot_doubles = [](int R) { return adj_slot_doubles<K>(R); };
      return l;
    }();
    return &L;
  }
  if (prec == 1) {
    static const Launchers L = make_fwd_launchers<Fwd<D, N, PDET, float>>();
    return &L;
  }
  if (prec == 2) {
    if constexpr (bf16_instantiated<PDET, D, N>()) {
      static const Launchers L = make_fwd_launchers<Fwd<D, N, PDET, float, false, true>>();
      return &L;
    }
  }
  return nullptr;
}

template <template <int> class PDET, int D, int... Ns>
const Launchers* pick_order(int order, int prec, bool st) {
  const Launchers* r = nullptr;
  ((order == Ns ? (r = pick_precision<PDET, D, Ns>(prec, st), 0) : 0), ...);
  return r;
}

}  // namespace adg
