// Shared compile-time helpers, table structs and launch arguments.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cmath>
#include <cstring>
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
  // Even/odd split of D, which is centro-antisymmetric on the symmetric
  // Gauss-Legendre nodes (D[n-1-k][n-1-j] = -D[k][j]); for k, j < n/2:
  // Ce = (D[k][j] + D[k][n-1-j]) / 2, Co = (D[k][j] - D[k][n-1-j]) / 2, and for
  // odd n the middle column Cm[k] = D[k][n/2] and middle row Dm[j] = D[n/2][j].
  static constexpr int H = n / 2 > 0 ? n / 2 : 1;
  Real Ce[H][H], Co[H][H], Cm[H], Dm[H];
  // bfloat16 pair of D for the matrix-core contraction: Dh = bf16(fl32(D)),
  // Dl = bf16(fl32(D - Dh)), both round to nearest even (bit patterns); their
  // sum is a 16-bit-significand operator that float32 holds exactly.
  uint16_t Dh[n][n], Dl[n][n];
  float Dx[n][n];   // Dh + Dl as a float (exact)
  // Power form of the linear predictor: beta[k-1] = w . P^(k-1) Ps for
  // k = 1..BK, from the (Real-rounded) P and Ps as the device used to
  // recompute them.  L^k u vanishes for k > d N (a degree-N polynomial per
  // axis, piecewise-constant material), so BK = 3 n + 3 terms cover every R.
  static constexpr int BK = 3 * n + 3;
  double beta[BK];
};

// float -> bfloat16 bit pattern, round to nearest, ties to even (finite x).
inline uint16_t bf16_bits_rne(float x) {
  uint32_t b;
  std::memcpy(&b, &x, 4);
  b += 0x7FFFu + ((b >> 16) & 1u);
  return (uint16_t)(b >> 16);
}
inline double bf16_bits_value(uint16_t h) {
  const uint32_t b = (uint32_t)h << 16;
  float f;
  std::memcpy(&f, &b, 4);
  return (double)f;
}

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
  for (int k = 0; k < n / 2; ++k) {
    for (int j = 0; j < n / 2; ++j) {
      t.Ce[k][j] = (Real)(0.5 * (h.D[k * n + j] + h.D[k * n + (n - 1 - j)]));
      t.Co[k][j] = (Real)(0.5 * (h.D[k * n + j] - h.D[k * n + (n - 1 - j)]));
    }
    t.Cm[k] = (Real)h.D[k * n + n / 2];
    t.Dm[k] = (Real)h.D[(n / 2) * n + k];
  }
  for (int k = 0; k < n; ++k)
    for (int j = 0; j < n; ++j) {
      const double d = h.D[k * n + j];
      t.Dh[k][j] = bf16_bits_rne((float)d);
      t.Dl[k][j] = bf16_bits_rne((float)(d - bf16_bits_value(t.Dh[k][j])));
      t.Dx[k][j] = (float)(bf16_bits_value(t.Dh[k][j]) + bf16_bits_value(t.Dl[k][j]));
    }
  {
    double T[n], Tn[n];
    for (int a = 0; a < n; ++a) T[a] = (double)t.Ps[a];
    for (int k = 1; k <= KTab<n, Real>::BK; ++k) {
      if (k > 1) {
        for (int a = 0; a < n; ++a) {
          double s = 0.0;
          for (int j = 0; j < n; ++j) s = std::fma((double)t.P[a][j], T[j], s);
          Tn[a] = s;
        }
        for (int a = 0; a < n; ++a) T[a] = Tn[a];
      }
      double b = 0.0;
      for (int a = 0; a < n; ++a) b = std::fma(t.w[a], T[a], b);
      t.beta[k - 1] = b;
    }
  }
  return t;
}

// Matrix-core contraction of a pencil (gfx950 v_mfma_f32_16x16x32_bf16).
// Operand layout of that instruction (verified on the device): lane l holds
// A[l % 16][8 (l / 16) + r] and B[8 (l / 16) + r][l % 16] in its register r
// (r < 8) and receives C[4 (l / 16) + i][l % 16] (i < 4).  With A block
// diagonal, A[4 g + i][8 g + j] = R_i[j] for lane group g = l / 16, each
// lane's 8 B values (its own pencil's inputs x_j, j < n) produce
// sum_j R_i[j] x_j, i < 4, in its own C: a per-lane contraction against four
// operator rows R_0..R_3.  Nodes 0..3 take two instructions (rows of Dh, then
// rows of Dl accumulated); nodes 4..n-1 one more when n <= 6 (rows
// Dh[4..n-1] and Dl[4..n-1] side by side, summed afterwards) and two when
// n > 6.  Every lane of the wave takes part; lanes without a task must hold
// finite inputs.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

template <int n>
struct MxOps {
  static constexpr int NH = n > 4 ? 2 : 1;          // output halves
  static constexpr bool PACK1 = n > 4 && n <= 6;    // second half: Dh and Dl rows in one operand
  bf16x8 hi[NH], lo[NH];                            // lo[1] unused when PACK1
};

template <int n, class Tab>
__device__ __forceinline__ MxOps<n> make_mx_ops(const Tab& t) {
  static_assert(n <= 8, "the matrix-core contraction takes at most 8 nodes per pencil");
  MxOps<n> o;
  const int l = (int)(threadIdx.x & 63);
  const int m = l & 15, g = l >> 4;
  const bool mine = (m >> 2) == g;
  // Rows are picked by selects over static indices: indexing the table by a
  // lane-dependent row makes the compiler copy the whole kernel argument
  // block to scratch memory at larger n.
#pragma unroll
  for (int h = 0; h < MxOps<n>::NH; ++h) {
    const int row = 4 * h + (m & 3);
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      uint16_t bh = 0, bl = 0;
      if (r < n) {
#pragma unroll
        for (int rr = 4 * h; rr < 4 * h + 4 && rr < n; ++rr) {
          bh = (row == rr) ? t.Dh[rr][r] : bh;
          bl = (row == rr) ? t.Dl[rr][r] : bl;
        }
      }
      if (!mine) bh = bl = 0;
      o.hi[h][r] = __builtin_bit_cast(__bf16, bh);
      o.lo[h][r] = __builtin_bit_cast(__bf16, bl);
    }
  }
  if constexpr (MxOps<n>::PACK1) {
    // rows i < n - 4: Dh[4 + i]; rows n - 4 <= i < 2 (n - 4): Dl[4 + i - (n - 4)]
    const int i = m & 3;
    const bool hi_row = i < n - 4, lo_row = i >= n - 4 && i < 2 * (n - 4);
    const int row = 4 + (hi_row ? i : (lo_row ? i - (n - 4) : 0));
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const bool on = mine && r < n && (hi_row || lo_row);
      const int rr = r < n ? r : 0;
      const uint16_t b = on ? (hi_row ? t.Dh[row][rr] : t.Dl[row][rr]) : (uint16_t)0;
      o.hi[1][r] = __builtin_bit_cast(__bf16, b);
    }
  }
  return o;
}

// The reference flux of a pencil: the first node for n < 5, the middle node
// for odd n, the mean of the middle pair for even n (computed in float as
// 0.5 (a + b)).
template <int n, int M>
__device__ __forceinline__ float pencil_ref(const float (&F)[n][M], int v) {
  if constexpr (n < 5) return F[0][v];
  else if constexpr (n % 2 == 1) return F[n / 2][v];
  else return 0.5f * (F[n / 2 - 1][v] + F[n / 2][v]);
}

// out[k][v] = sum_j D[k][j] x_j[v] with x_j = bf16(F_j - F_ref) (round to
// nearest even) and D = Dh + Dl, float32 accumulation on the matrix cores.
template <int n, int M, class FluxAt>
__device__ __forceinline__ void pencil_dF_mx(const MxOps<n>& A, FluxAt&& flux_at,
                                             float (&out)[n][M]) {
  float F[n][M];
#pragma unroll
  for (int j = 0; j < n; ++j) flux_at(j, F[j]);
  constexpr int jr = (n < 5) ? 0 : ((n % 2 == 1) ? n / 2 : -1);   // x_jr = 0 exactly
#pragma unroll
  for (int v = 0; v < M; ++v) {
    const float Fr = pencil_ref<n, M>(F, v);
    bf16x8 B;
#pragma unroll
    for (int r = 0; r < 8; ++r)
      B[r] = (r < n && r != jr) ? (__bf16)(F[r < n ? r : 0][v] - Fr) : (__bf16)0.0f;
    floatx4 c = {0.0f, 0.0f, 0.0f, 0.0f};
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A.hi[0], B, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A.lo[0], B, c, 0, 0, 0);
#pragma unroll
    for (int i = 0; i < 4; ++i)
      if (i < n) out[i][v] = c[i];
    if constexpr (MxOps<n>::PACK1) {
      floatx4 e = {0.0f, 0.0f, 0.0f, 0.0f};
      e = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A.hi[1], B, e, 0, 0, 0);
#pragma unroll
      for (int i = 0; i < n - 4; ++i) out[4 + i][v] = e[i] + e[i + (n - 4)];
    } else if constexpr (MxOps<n>::NH == 2) {
      floatx4 e = {0.0f, 0.0f, 0.0f, 0.0f};
      e = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A.hi[1], B, e, 0, 0, 0);
      e = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A.lo[1], B, e, 0, 0, 0);
#pragma unroll
      for (int i = 0; i < 4; ++i)
        if (4 + i < n) out[4 + i][v] = e[i];
    }
  }
}

// One pencil's contraction out[k][v] = sum_j D[k][j] F_j[v], F_j from
// flux_at(j, F).  For n >= 5 the even/odd split of the centro-antisymmetric D
// halves the multiplications: with E_j = F_j + F_{n-1-j} and
// O_j = F_j - F_{n-1-j}, for k, j < n/2
//   out[k] = S_k + A_k, out[n-1-k] = A_k - S_k, out[n/2] = sum_j Dm[j] O_j,
//   S_k = sum_j Ce[k][j] E_j + Cm[k] F_{n/2} (odd n), A_k = sum_j Co[k][j] O_j.
// float: the rounded coefficients no longer sum to zero along a row, so a
// constant flux would get a derivative of float rounding size.  The float
// forms therefore contract against a reference flux F_r, which the zero row
// sums of D allow: n < 5 subtracts F_0; the split takes E_j - 2 F_r with F_r
// the middle node (odd n, which removes the Cm column) or the middle pair's
// mean (even n, whose even term then drops).  A constant flux then gives
// exactly zero.  float64 keeps the plain forms (its rounding is float64's).
template <int n, int M, class Real, class Tab, class FluxAt>
__device__ __forceinline__ void pencil_dF(const Tab& t, FluxAt&& flux_at, Real (&out)[n][M]) {
  constexpr bool REF = !std::is_same<Real, double>::value;
  if constexpr (n < 5) {
    Real F0[M];
#pragma unroll
    for (int k = 0; k < n; ++k)
#pragma unroll
      for (int v = 0; v < M; ++v) out[k][v] = Real(0);
    if constexpr (REF) flux_at(0, F0);
#pragma unroll
    for (int j = REF ? 1 : 0; j < n; ++j) {
      Real F[M];
      flux_at(j, F);
#pragma unroll
      for (int v = 0; v < M; ++v) {
        const Real G = REF ? F[v] - F0[v] : F[v];
#pragma unroll
        for (int k = 0; k < n; ++k) out[k][v] = fma(t.D[k][j], G, out[k][v]);
      }
    }
  } else {
    constexpr int h = n / 2;
    constexpr bool odd = (n % 2) == 1;
    Real S[h][M], A[h][M], Mid[M];
#pragma unroll
    for (int v = 0; v < M; ++v) {
      Mid[v] = Real(0);
#pragma unroll
      for (int k = 0; k < h; ++k) S[k][v] = A[k][v] = Real(0);
    }
    if constexpr (!REF) {
#pragma unroll
      for (int j = 0; j < h; ++j) {
        Real Fa[M], Fb[M];
        flux_at(j, Fa);
        flux_at(n - 1 - j, Fb);
#pragma unroll
        for (int v = 0; v < M; ++v) {
          const Real E = Fa[v] + Fb[v], O = Fa[v] - Fb[v];
#pragma unroll
          for (int k = 0; k < h; ++k) {
            S[k][v] = fma(t.Ce[k][j], E, S[k][v]);
            A[k][v] = fma(t.Co[k][j], O, A[k][v]);
          }
          if constexpr (odd) Mid[v] = fma(t.Dm[j], O, Mid[v]);
        }
      }
      if constexpr (odd) {
        Real Fm[M];
        flux_at(h, Fm);
#pragma unroll
        for (int k = 0; k < h; ++k)
#pragma unroll
          for (int v = 0; v < M; ++v) S[k][v] = fma(t.Cm[k], Fm[v], S[k][v]);
      }
    } else {
      Real Er[M];                                  // 2 F_r
      if constexpr (odd) {
        Real Fm[M];
        flux_at(h, Fm);
#pragma unroll
        for (int v = 0; v < M; ++v) Er[v] = Real(2) * Fm[v];
      } else {
        Real Fa[M], Fb[M];                         // the middle pair: its E is 2 F_r
        flux_at(h - 1, Fa);
        flux_at(h, Fb);
#pragma unroll
        for (int v = 0; v < M; ++v) {
          Er[v] = Fa[v] + Fb[v];
          const Real O = Fa[v] - Fb[v];
#pragma unroll
          for (int k = 0; k < h; ++k) A[k][v] = fma(t.Co[k][h - 1], O, A[k][v]);
        }
      }
#pragma unroll
      for (int j = 0; j < (odd ? h : h - 1); ++j) {
        Real Fa[M], Fb[M];
        flux_at(j, Fa);
        flux_at(n - 1 - j, Fb);
#pragma unroll
        for (int v = 0; v < M; ++v) {
          const Real E = (Fa[v] + Fb[v]) - Er[v], O = Fa[v] - Fb[v];
#pragma unroll
          for (int k = 0; k < h; ++k) {
            S[k][v] = fma(t.Ce[k][j], E, S[k][v]);
            A[k][v] = fma(t.Co[k][j], O, A[k][v]);
          }
          if constexpr (odd) Mid[v] = fma(t.Dm[j], O, Mid[v]);
        }
      }
    }
#pragma unroll
    for (int k = 0; k < h; ++k)
#pragma unroll
      for (int v = 0; v < M; ++v) {
        out[k][v] = S[k][v] + A[k][v];
        out[n - 1 - k][v] = A[k][v] - S[k][v];
      }
    if constexpr (odd) {
#pragma unroll
      for (int v = 0; v < M; ++v) out[h][v] = Mid[v];
    }
  }
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
  bool traces_only = false;         // predictor: hull only, no Q~ (adjoint replay)
  double* st_face = nullptr;        // space-time corrector: F* of the lower faces
  double* adj_tb = nullptr;         // adjoint: trace bars
  double* adj_slots = nullptr;      // adjoint: per-block Picard scratch
  double* adj_pf = nullptr;         // adjoint: per (cell, face) material bars
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
  LaunchFn fv_project = nullptr;       // subcell patches of the limiter (float64)
  LaunchFn fv_reconstruct = nullptr;
  LaunchFn fv_step = nullptr;
  int64_t trace_bytes_per_cell = 0;
  int64_t qdofs_per_cell = 0;                  // m (N+1)^d
  int64_t adj_pf_per_cell = 0;                 // 2d NPAR (adjoint face material bars)
  int64_t st_face_per_cell = 0;                // d (N+1)^(d-1) m (space-time corrector)
  int64_t (*adj_slot_doubles)(int R) = nullptr;
};

// Registries implemented by the per-PDE instantiation units.
const Launchers* find_advection(int dim, int order, int prec, bool st);
const Launchers* find_euler(int dim, int order, int prec, bool st);
const Launchers* find_acoustic(int dim, int order, int prec, bool st);
const Launchers* find_elastic(int dim, int order, int prec, bool st);

// Grid size used by every cell-parallel reduction kernel (partial maxima).
constexpr int64_t kMaxReduceBlocks = 16384;

}  // namespace adg
