// Shared compile-time helpers, table structs and launch arguments.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "pde.hpp"
#include "tables.hpp"

namespace adg {

constexpr int ipow(int b, int e) { return e == 0 ? 1 : b * ipow(b, e - 1); }

template <int B, int E, class F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}

// Node index of point j of the pencil along axis I through face node b
// (b enumerates the other coordinates, lower axes fastest).
template <int n, int I>
__device__ __forceinline__ int pencil_node(int b, int j) {
  constexpr int s = ipow(n, I);
  return (b % s) + s * (j + n * (b / s));
}

// Face node index (of the face normal to axis I) of spatial node a.
template <int n, int I>
__device__ __forceinline__ int face_node(int a) {
  constexpr int s = ipow(n, I);
  return (a % s) + s * (a / (s * n));
}

// Coordinate I of spatial node a.
template <int n, int I>
__device__ __forceinline__ int coord(int a) {
  return (a / ipow(n, I)) % n;
}

// 1D operators passed by value (kernel arguments live in the constant
// kernarg segment; uniform loads land in scalar registers).
template <int n, class Real>
struct KTab {
  Real D[n][n];     // derivative matrix (Picard contractions)
  Real P[n][n];     // Picard time operator
  Real Ps[n];       // row sums of P (time operator applied to a constant)
  double w[n];      // GL weights (time averages)
  double Kv[n][n];  // volume operator
  double FL[n], FR[n], LL[n], LR[n];
};

template <int n, class Real>
inline KTab<n, Real> make_ktab(const HostTables& h) {
  KTab<n, Real> t;
  for (int a = 0; a < n; ++a) {
    double ps = 0.0;
    t.w[a] = h.w[a];
    t.FL[a] = h.FL[a];
    t.FR[a] = h.FR[a];
    t.LL[a] = h.LL[a];
    t.LR[a] = h.LR[a];
    for (int j = 0; j < n; ++j) {
      t.D[a][j] = (Real)h.D[a * n + j];
      t.P[a][j] = (Real)h.P[a * n + j];
      ps += h.P[a * n + j];
      t.Kv[a][j] = h.Kv[a * n + j];
    }
    t.Ps[a] = (Real)ps;
  }
  return t;
}

// Everything a launcher needs from the context.
struct LaunchArgs {
  double* Q = nullptr;
  // Optional separate input / output of the predictor and corrector (both
  // default to Q in place) and, for the fused step, the hull it writes, the
  // predictor's time step and the rerun switch.
  const double* qin = nullptr;
  double* qout = nullptr;
  void* traces_out = nullptr;
  const double* dt_pred = nullptr;
  const int32_t* run_if = nullptr;
  const double* Qc = nullptr;       // read-only state (wave speed / adjoint)
  const double* params = nullptr;
  const double* dt = nullptr;
  double* Qbar = nullptr;           // adjoint in/out
  double* params_bar = nullptr;     // adjoint accumulator
  int32_t* flag = nullptr;
  void* traces = nullptr;           // face hull
  double* adj_qtmp = nullptr;       // adjoint: copy of Q for the traces
  double* adj_tb = nullptr;         // adjoint: trace bars
  double* adj_slots = nullptr;      // adjoint: per-block Picard scratch
  int64_t adj_nslots = 0;
  double* partial = nullptr;        // per-block maxima
  int64_t n_partial = 0;            // capacity of partial
  int64_t* n_partial_used = nullptr;// host-side record of the last count
  int64_t ncells = 0;
  int nc[3] = {1, 1, 1};
  int brick[3] = {1, 1, 1};         // brick walk of the corrector
  double inv_h = 1.0;
  int R = 1;
  double gp[4] = {0, 0, 0, 0};      // global PDE constants (see pde.hpp)
  const HostTables* tab = nullptr;
  hipStream_t stream = nullptr;
};

using LaunchFn = int (*)(const LaunchArgs&);   // returns 0 or a hipError_t

struct Launchers {
  LaunchFn predict = nullptr;
  LaunchFn correct = nullptr;
  LaunchFn wave_speed = nullptr;
  LaunchFn adjoint = nullptr;
  LaunchFn fused = nullptr;
  int64_t trace_bytes_per_cell = 0;
  int64_t qdofs_per_cell = 0;                  // m (N+1)^d
  int64_t (*adj_slot_doubles)(int R) = nullptr;
};

// Registries implemented by the per-PDE instantiation units.
const Launchers* find_advection(int dim, int order, int prec);
const Launchers* find_euler(int dim, int order, int prec);
const Launchers* find_acoustic(int dim, int order, int prec);
const Launchers* find_elastic(int dim, int order, int prec);

// Grid size used by every cell-parallel reduction kernel (partial maxima).
constexpr int64_t kMaxReduceBlocks = 16384;

}  // namespace adg
