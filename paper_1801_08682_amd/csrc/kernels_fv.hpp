// Finite-volume subcell patches of the limiter (Sec. 3, "Finite Volume
// limiter"; App. A, Corollary 8) for gfx950.
//
// Every cell of order N carries S^d subcells, S = 2N + 1, as
// P[cell][subcell][var] (subcells lexicographic, x fastest).  The subgrid
// step is first-order finite volumes with Rusanov fluxes, i.e. ADER-DG with
// p = 0 on the subgrid: the predictor is the identity and a subcell's face
// traces are its own value and flux (Corollary 8), so the corrector of a
// subcell reads its 2d face neighbours' states directly (one kernel, the
// traces never stored):
//   Q <- Q - (dt S / h) sum_i (F*_{i,+} - F*_{i,-}),
//   F* = (f_L + f_R) / 2 - s (Q_R - Q_L) / 2, s = max(lambda_L, lambda_R).
// Both subcells of a face evaluate its flux with the same operands in the
// same order, so the totals are conserved to round-off.  A subcell's
// material is its cell's.
//
//  k_fv_project      DG nodal values -> subcell averages (Pi per axis)
//  k_fv_reconstruct  subcell averages -> DG nodal values (least squares, Rc)
//  k_fv_step         one Rusanov step on the subgrid, out of place, plus the
//                    per-block wave-speed maxima of the new state and the flag
#pragma once

#include "kernels_fwd.hpp"

namespace adg {

template <class K>
struct FvP {
  static constexpr int n = K::n, S = 2 * K::N + 1;
  const double* in;      // Q (project) or P (reconstruct, step)
  double* out;           // P (project, step) or Q (reconstruct)
  const double* par;
  const double* dt;
  double* partial;       // step: per-block maxima of the new state's speeds
  int32_t* flag;
  int64_t ncells;
  int nc[3];
  double inv_hs;         // S / h
  Gconst<double> g;
  double Pi[S][n];       // subcell averages of the Lagrange basis
  double Rc[n][S];       // least-squares reconstruction
};

// out[c][o][v] = sum_{i_0..i_{d-1}} prod_a M[o_a][i_a] in[c][i][v]: a direct
// tensor-product contraction, one thread per (cell, output point).
template <class K, int EO, int EI, class Mat>
__device__ __forceinline__ void tensor_apply(const FvP<K>& p, const Mat& Mx, int64_t gid) {
  constexpr int D = K::D, M = K::M, NO = ipow(EO, D), NI = ipow(EI, D);
  const int64_t cell = gid / NO;
  const int o = (int)(gid - cell * NO);
  double acc[M];
#pragma unroll
  for (int v = 0; v < M; ++v) acc[v] = 0.0;
  int oc[D];
#pragma unroll
  for (int a = 0; a < D; ++a) oc[a] = (o / ipow(EO, a)) % EO;
  const double* src = p.in + cell * NI * M;
  for (int i = 0; i < NI; ++i) {
    double w = 1.0;
#pragma unroll
    for (int a = 0; a < D; ++a) w *= Mx[oc[a]][(i / ipow(EI, a)) % EI];
#pragma unroll
    for (int v = 0; v < M; ++v) acc[v] = fma(w, src[i * M + v], acc[v]);
  }
  double* dst = p.out + (cell * NO + o) * M;
#pragma unroll
  for (int v = 0; v < M; ++v) dst[v] = acc[v];
}

template <class K>
__global__ void __launch_bounds__(256) k_fv_project(const FvP<K> p) {
  constexpr int NO = ipow(FvP<K>::S, K::D);
  const int64_t total = p.ncells * NO;
  for (int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x; g < total; g += (int64_t)gridDim.x * 256)
    tensor_apply<K, FvP<K>::S, K::n>(p, p.Pi, g);
}

template <class K>
__global__ void __launch_bounds__(256) k_fv_reconstruct(const FvP<K> p) {
  constexpr int NO = ipow(K::n, K::D);
  const int64_t total = p.ncells * NO;
  for (int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x; g < total; g += (int64_t)gridDim.x * 256)
    tensor_apply<K, K::n, FvP<K>::S>(p, p.Rc, g);
}

// Global subcell index of the face neighbour of subcell (cell, sc) along axis
// I in direction dir (periodic over the whole subgrid).
template <class K, int I>
__device__ __forceinline__ int64_t fv_neighbour(int64_t cell, int sc, int dir, const int* nc) {
  constexpr int S = FvP<K>::S, NSC = ipow(S, K::D), sI = ipow(S, I);
  const int k = (sc / sI) % S;
  int kn = k + dir;
  int64_t cn = cell;
  if (kn < 0 || kn >= S) {
    kn = kn < 0 ? S - 1 : 0;
    cn = neighbour<K>(cell, I, dir, nc);
  }
  return cn * NSC + sc + (kn - k) * sI;
}

// Rusanov flux along +e_I between the states qL (left) and qR (right).
template <class K, int I>
__device__ __forceinline__ void fv_flux(const FvP<K>& p, const double* qL, const double* qR,
                                        const typename K::PDE::template CP<double>& cL,
                                        const typename K::PDE::template CP<double>& cR,
                                        double* Fs, bool& bad) {
  using PDE = typename K::PDE;
  constexpr int M = K::M;
  double fL[M], fR[M];
  PDE::template flux<I>(qL, fL, p.g, cL);
  PDE::template flux<I>(qR, fR, p.g, cR);
  const double s = fmax(PDE::template speed<I>(qL, p.g, cL), PDE::template speed<I>(qR, p.g, cR));
  if (!(s >= 0.0)) bad = true;
#pragma unroll
  for (int v = 0; v < M; ++v) Fs[v] = 0.5 * (fL[v] + fR[v]) - 0.5 * s * (qR[v] - qL[v]);
}

template <class K>
__global__ void __launch_bounds__(256) k_fv_step(const FvP<K> p) {
  using PDE = typename K::PDE;
  constexpr int D = K::D, M = K::M, NPAR = K::NPAR;
  constexpr int NSC = ipow(FvP<K>::S, D);
  __shared__ double red[4];
  const int64_t total = p.ncells * NSC;
  const double c = (*p.dt) * p.inv_hs;
  double lmax = 0.0;
  int bad = 0;
  for (int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x; g < total; g += (int64_t)gridDim.x * 256) {
    const int64_t cell = g / NSC;
    const int sc = (int)(g - cell * NSC);
    double q[M], qn[M];
#pragma unroll
    for (int v = 0; v < M; ++v) qn[v] = q[v] = p.in[g * M + v];
    const auto cp = PDE::template cell<double>(p.par + cell * NPAR);
    bool badf = false;
    static_for<0, D>([&](auto I_) {
      constexpr int I = decltype(I_)::value;
      const int64_t gm = fv_neighbour<K, I>(cell, sc, -1, p.nc);
      const int64_t gp = fv_neighbour<K, I>(cell, sc, +1, p.nc);
      double qm[M], qp[M], Fm[M], Fp[M];
#pragma unroll
      for (int v = 0; v < M; ++v) {
        qm[v] = p.in[gm * M + v];
        qp[v] = p.in[gp * M + v];
      }
      const auto cm = PDE::template cell<double>(p.par + (gm / NSC) * NPAR);
      const auto cq = PDE::template cell<double>(p.par + (gp / NSC) * NPAR);
      fv_flux<K, I>(p, qm, q, cm, cp, Fm, badf);   // left face: (left neighbour, self)
      fv_flux<K, I>(p, q, qp, cp, cq, Fp, badf);   // right face: (self, right neighbour)
#pragma unroll
      for (int v = 0; v < M; ++v) qn[v] -= c * (Fp[v] - Fm[v]);
    });
#pragma unroll
    for (int v = 0; v < M; ++v) p.out[g * M + v] = qn[v];
    static_for<0, D>([&](auto I_) {
      constexpr int I = decltype(I_)::value;
      lmax = fmax(lmax, PDE::template speed<I>(qn, p.g, cp));
    });
    if (badf) bad |= 2;
    if (!PDE::admissible(qn, p.g, cp)) {
      bool fin = true;
#pragma unroll
      for (int v = 0; v < M; ++v) fin = fin && isfinite(qn[v]);
      bad |= fin ? 2 : 1;
    }
  }
  const double bm = block_max<256>(lmax, red);
  if (threadIdx.x == 0) p.partial[blockIdx.x] = bm;
  if (bad && p.flag) atomicOr(p.flag, bad);
}

template <class K>
FvP<K> fv_params(const LaunchArgs& a) {
  FvP<K> p;
  constexpr int n = K::n, S = FvP<K>::S;
  p.par = a.params;
  p.dt = a.dt;
  p.partial = a.partial;
  p.flag = a.flag;
  p.ncells = a.ncells;
  for (int k = 0; k < 3; ++k) p.nc[k] = a.nc[k];
  p.inv_hs = a.inv_h * S;
  for (int k = 0; k < 4; ++k) p.g.c[k] = a.gp[k];
  for (int sc = 0; sc < S; ++sc)
    for (int j = 0; j < n; ++j) {
      p.Pi[sc][j] = a.tab->Pi[sc * n + j];
      p.Rc[j][sc] = a.tab->Rc[j * S + sc];
    }
  return p;
}

// Grid-stride launches over at most kMaxReduceBlocks blocks of 256 threads.
inline int64_t fv_blocks(int64_t items) {
  int64_t G = (items + 255) / 256;
  return G < kMaxReduceBlocks ? (G > 0 ? G : 1) : kMaxReduceBlocks;
}

// a.qin -> a.qout for every launcher below.
template <class K>
int launch_fv_project(const LaunchArgs& a) {
  FvP<K> p = fv_params<K>(a);
  p.in = a.qin;
  p.out = a.qout;
  const int64_t G = fv_blocks(a.ncells * ipow(FvP<K>::S, K::D));
  hipLaunchKernelGGL(k_fv_project<K>, dim3((unsigned)G), dim3(256), 0, a.stream, p);
  return (int)hipGetLastError();
}

template <class K>
int launch_fv_reconstruct(const LaunchArgs& a) {
  FvP<K> p = fv_params<K>(a);
  p.in = a.qin;
  p.out = a.qout;
  const int64_t G = fv_blocks(a.ncells * K::NS);
  hipLaunchKernelGGL(k_fv_reconstruct<K>, dim3((unsigned)G), dim3(256), 0, a.stream, p);
  return (int)hipGetLastError();
}

template <class K>
int launch_fv_step(const LaunchArgs& a) {
  FvP<K> p = fv_params<K>(a);
  p.in = a.qin;
  p.out = a.qout;
  const int64_t G = fv_blocks(a.ncells * ipow(FvP<K>::S, K::D));
  if (G > a.n_partial) return (int)hipErrorInvalidValue;
  *a.n_partial_used = G;
  hipLaunchKernelGGL(k_fv_step<K>, dim3((unsigned)G), dim3(256), 0, a.stream, p);
  return (int)hipGetLastError();
}

}  // namespace adg
