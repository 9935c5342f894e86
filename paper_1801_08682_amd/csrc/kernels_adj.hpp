// Reverse mode (discrete adjoint) of one ADER-DG step, dt held fixed.
//
// The step is Q+ = Q~ - (dt/h) sum_i (LR F*_{i,+} - LL F*_{i,-}) with
// Q~ = u + (dt/h) V(Fbar), traces from the Picard predictor q^R (Sec. 3,
// Eq. (2)-(6)).  Given G = dJ/dQ+:
//
//  k_adj_corr  per cell and face: the face-flux bar
//                Fb* = -(dt/h) LR^T G(left cell) + (dt/h) LL^T G(right cell),
//              its Rusanov transpose (qL, qR, fL, fR bars; the maximum speed
//              s passes its bar to the first maximal face node, left side
//              first), written as this cell's own trace bars.  Both cells of
//              a face compute the face quantities identically; each writes
//              only its own bars and material bars (no atomics).
//  k_adj_pred  per cell: recompute the Picard iterates q^0..q^R into a
//              per-block scratch slot, map the trace bars and Kv^T G back to
//              bars of (qbar, Fbar_i), then sweep the iterations backwards:
//              rhs bar = -(dt/h) P^T qb, F_i bar = D_i^T rhs bar,
//              q^{r-1} bar = sum_i J_i(q^{r-1})^T F_i bar, u bar += sum_t q^r bar.
#pragma once

#include "kernels_fwd.hpp"

namespace adg {

template <class K>
struct AdjCorrP {
  const double* G;       // dJ/dQ+ (cell, node, var)
  const double* par;
  const double* dt;
  const double* tr;      // forward traces of Q (float64)
  double* tb;            // trace bars, same layout as the traces
  double* pbar;          // per-cell material bars (nullable)
  int64_t ncells;
  int nc[3];
  double inv_h;
  Gconst<double> g;
  double LL[K::n], LR[K::n];
};

template <class K>
__global__ void __launch_bounds__(K::CT) k_adj_corr(const AdjCorrP<K> p) {
  using PDE = typename K::PDE;
  constexpr int n = K::n, M = K::M, NF = K::NF, D = K::D, CT = K::CT, NPAR = K::NPAR;
  constexpr int FT = 2 * D * NF;
  __shared__ double lamL[FT], lamR[FT], sbp[FT];
  __shared__ double smax[2 * D], sbar[2 * D];
  __shared__ int bstar[2 * D], sstar[2 * D];
  __shared__ double pred[NPAR > 0 ? NPAR * CT : 1];
  const int t = threadIdx.x;
  const double cdt = (*p.dt) * p.inv_h;

  for (GroupIter it(p.ncells); it.g < it.end; it.g += it.step) {
    const int64_t cell = it.g;
    double pb[NPAR > 0 ? NPAR : 1];
#pragma unroll
    for (int k = 0; k < (NPAR > 0 ? NPAR : 1); ++k) pb[k] = 0.0;
    double qL[M], qR[M], Fb[M], dq[M];
    int f = 0, b = 0, i = 0, s = 0;
    int64_t cL = 0, cR = 0;
    const bool ftask = t < FT;
    if (ftask) {
      f = t / NF;
      b = t - f * NF;
      i = f >> 1;
      s = f & 1;
      cL = s ? cell : neighbour<K>(cell, i, -1, p.nc);
      cR = s ? neighbour<K>(cell, i, +1, p.nc) : cell;
      const double* trL = p.tr + cL * K::TRACE_ELEMS + (int64_t)(2 * i + 1) * K::NQ * NF * M + b * M;
      const double* trR = p.tr + cR * K::TRACE_ELEMS + (int64_t)(2 * i) * K::NQ * NF * M + b * M;
#pragma unroll
      for (int v = 0; v < M; ++v) {
        qL[v] = trL[v];
        qR[v] = trR[v];
        dq[v] = qR[v] - qL[v];
        Fb[v] = 0.0;
      }
      const auto pL = PDE::template cell<double>(p.par + cL * NPAR);
      const auto pR = PDE::template cell<double>(p.par + cR * NPAR);
      static_for<0, D>([&](auto I_) {
        constexpr int I = decltype(I_)::value;
        if (i == I) {
          lamL[t] = PDE::template speed<I>(qL, p.g, pL);
          lamR[t] = PDE::template speed<I>(qR, p.g, pR);
          // Fb* = -(dt/h) (LR^T G_L)_b + (dt/h) (LL^T G_R)_b
          const double* GL = p.G + cL * K::NS * M;
          const double* GR = p.G + cR * K::NS * M;
#pragma unroll
          for (int k = 0; k < n; ++k) {
            const int nd = pencil_node<n, I>(b, k);
#pragma unroll
            for (int v = 0; v < M; ++v)
              Fb[v] += -cdt * p.LR[k] * GL[nd * M + v] + cdt * p.LL[k] * GR[nd * M + v];
          }
        }
      });
      double sp = 0.0;
#pragma unroll
      for (int v = 0; v < M; ++v) sp += Fb[v] * dq[v];
      sbp[t] = -0.5 * sp;
    }
    __syncthreads();
    if (t < 2 * D) {
      double best = -1.0, acc = 0.0;
      int bs = 0, ss = 0;
      for (int bb = 0; bb < NF; ++bb) {
        const double l0 = lamL[t * NF + bb], l1 = lamR[t * NF + bb];
        if (l0 > best) { best = l0; bs = bb; ss = 0; }
        if (l1 > best) { best = l1; bs = bb; ss = 1; }
        acc += sbp[t * NF + bb];
      }
      smax[t] = best;
      bstar[t] = bs;
      sstar[t] = ss;
      sbar[t] = acc;
    }
    __syncthreads();
    if (ftask) {
      // this cell is the left state of its right face (s = 1) and the right
      // state of its left face (s = 0)
      double tq[M], tf[M];
      const double* own = s ? qL : qR;
      const double sgn = s ? 0.5 : -0.5;
#pragma unroll
      for (int v = 0; v < M; ++v) {
        tq[v] = sgn * smax[f] * Fb[v];
        tf[v] = 0.5 * Fb[v];
      }
      const auto pc = PDE::template cell<double>(p.par + cell * NPAR);
      const bool mine = (bstar[f] == b) && (sstar[f] == (s ? 0 : 1));
      static_for<0, D>([&](auto I_) {
        constexpr int I = decltype(I_)::value;
        if (i == I) {
          if (mine) PDE::template speed_adj<I>(own, sbar[f], tq, pb, p.g, pc);
          if constexpr (K::NQ == 1) PDE::template flux_adj<I>(own, tf, tq, pb, p.g, pc);
        }
      });
      double* out = p.tb + cell * K::TRACE_ELEMS + (int64_t)f * K::NQ * NF * M + b * M;
#pragma unroll
      for (int v = 0; v < M; ++v) out[v] = tq[v];
      if constexpr (K::NQ == 2) {
#pragma unroll
        for (int v = 0; v < M; ++v) out[NF * M + v] = tf[v];
      }
    }
    if constexpr (NPAR > 0) {
#pragma unroll
      for (int k = 0; k < NPAR; ++k) pred[k * CT + t] = pb[k];
      __syncthreads();
      if (t < NPAR && p.pbar) {
        double acc = 0.0;
        for (int j = 0; j < CT; ++j) acc += pred[t * CT + j];
        p.pbar[cell * NPAR + t] += acc;
      }
    }
    __syncthreads();
  }
}

template <class K>
struct AdjPredP {
  const double* Q;       // Q(T)
  const double* par;
  const double* dt;
  double* Qbar;          // in: dJ/dQ+, out: dJ/dQ
  const double* tb;      // trace bars
  double* pbar;
  double* scratch;       // per-block slots
  int64_t slot_doubles;
  int64_t ncells;
  double inv_h;
  int R;
  Gconst<double> g;
  KTab<K::n, double> t;
};

template <class K>
constexpr int64_t adj_slot_doubles(int R) {
  // iterates q^0..q^R, fluxes of one iterate (d levels), rhs bar, iterate bar
  return (int64_t)((R + 1) + K::D + 2) * K::n * K::M * K::NS;
}

// One thread per spatial node; every space-time array lives in the block's
// scratch slot (L1/L2 resident) and each thread keeps only m-vectors.
template <class K>
__global__ void __launch_bounds__(K::NS) k_adj_pred(const AdjPredP<K> p) {
  using PDE = typename K::PDE;
  constexpr int n = K::n, M = K::M, NS = K::NS, NF = K::NF, D = K::D, NPAR = K::NPAR;
  constexpr int PL = n * M * NS;                 // one space-time level
  __shared__ double pred[NPAR > 0 ? NPAR * NS : 1];
  const int a = threadIdx.x;
  double* QI = p.scratch + (int64_t)blockIdx.x * p.slot_doubles;   // [R+1][n][M][NS]
  double* FS = QI + (int64_t)(p.R + 1) * PL;                         // [D][n][M][NS]
  double* RB = FS + (int64_t)D * PL;                                 // [n][M][NS]
  double* QB = RB + PL;                                              // [n][M][NS]
  const double c = (*p.dt) * p.inv_h;
  auto at = [](double* base, int tt, int v, int nd) -> double& { return base[(tt * M + v) * NS + nd]; };

  for (int64_t cell = blockIdx.x; cell < p.ncells; cell += gridDim.x) {
    double u[M];
#pragma unroll
    for (int v = 0; v < M; ++v) u[v] = p.Q[(cell * NS + a) * M + v];
    const auto cp = PDE::template cell<double>(p.par + cell * NPAR);
    double pb[NPAR > 0 ? NPAR : 1];
#pragma unroll
    for (int k = 0; k < (NPAR > 0 ? NPAR : 1); ++k) pb[k] = 0.0;

    // ---- recompute the Picard iterates (full iterations) ----
    for (int tt = 0; tt < n; ++tt)
#pragma unroll
      for (int v = 0; v < M; ++v) at(QI, tt, v, a) = u[v];
    for (int r = 1; r <= p.R; ++r) {
      const double* Qp = QI + (int64_t)(r - 1) * PL;
      for (int tt = 0; tt < n; ++tt) {
        double q[M];
#pragma unroll
        for (int v = 0; v < M; ++v) q[v] = Qp[(tt * M + v) * NS + a];
        static_for<0, D>([&](auto I_) {
          constexpr int I = decltype(I_)::value;
          double F[M];
          PDE::template flux<I>(q, F, p.g, cp);
#pragma unroll
          for (int v = 0; v < M; ++v) at(FS + I * PL, tt, v, a) = F[v];
        });
      }
      __syncthreads();
      for (int tt = 0; tt < n; ++tt) {
        double rhs[M];
#pragma unroll
        for (int v = 0; v < M; ++v) rhs[v] = 0.0;
        static_for<0, D>([&](auto I_) {
          constexpr int I = decltype(I_)::value;
          const int ai = coord<n, I>(a), fb = face_node<n, I>(a);
          for (int j = 0; j < n; ++j) {
            const int nd = pencil_node<n, I>(fb, j);
            const double dj = p.t.D[ai][j];
#pragma unroll
            for (int v = 0; v < M; ++v) rhs[v] += dj * at(FS + I * PL, tt, v, nd);
          }
        });
#pragma unroll
        for (int v = 0; v < M; ++v) at(RB, tt, v, a) = rhs[v];
      }
      double* Qr = QI + (int64_t)r * PL;
      for (int tt = 0; tt < n; ++tt)
#pragma unroll
        for (int v = 0; v < M; ++v) {
          double s = 0.0;
          for (int l = 0; l < n; ++l) s += p.t.P[tt][l] * at(RB, l, v, a);
          Qr[(tt * M + v) * NS + a] = u[v] - c * s;
        }
      __syncthreads();
    }

    // ---- bars of qbar and Fbar_i at this node ----
    const double* TB = p.tb + cell * K::TRACE_ELEMS;
    const double* Gc = p.Qbar + cell * NS * M;
    double qbb[M], Fbb[D][M];
#pragma unroll
    for (int v = 0; v < M; ++v) qbb[v] = 0.0;
    static_for<0, D>([&](auto I_) {
      constexpr int I = decltype(I_)::value;
      const int ai = coord<n, I>(a), fb = face_node<n, I>(a);
      const double* tl = TB + (int64_t)(2 * I) * K::NQ * NF * M + fb * M;
      const double* trr = TB + (int64_t)(2 * I + 1) * K::NQ * NF * M + fb * M;
#pragma unroll
      for (int v = 0; v < M; ++v) {
        qbb[v] += p.t.FL[ai] * tl[v] + p.t.FR[ai] * trr[v];
        Fbb[I][v] = (K::NQ == 2) ? p.t.FL[ai] * tl[NF * M + v] + p.t.FR[ai] * trr[NF * M + v] : 0.0;
      }
      for (int k = 0; k < n; ++k) {
        const int nd = pencil_node<n, I>(fb, k);
        const double kv = c * p.t.Kv[k][ai];
#pragma unroll
        for (int v = 0; v < M; ++v) Fbb[I][v] += kv * Gc[nd * M + v];
      }
    });
    {
      const double* QR = QI + (int64_t)p.R * PL;
      for (int tt = 0; tt < n; ++tt) {
        double q[M], acc[M];
        const double wt = p.t.w[tt];
#pragma unroll
        for (int v = 0; v < M; ++v) {
          q[v] = QR[(tt * M + v) * NS + a];
          acc[v] = wt * qbb[v];
        }
        static_for<0, D>([&](auto I_) {
          constexpr int I = decltype(I_)::value;
          double fw[M];
#pragma unroll
          for (int v = 0; v < M; ++v) fw[v] = wt * Fbb[I][v];
          PDE::template flux_adj<I>(q, fw, acc, pb, p.g, cp);
        });
#pragma unroll
        for (int v = 0; v < M; ++v) at(QB, tt, v, a) = acc[v];
      }
    }

    // ---- reverse sweep over the Picard iterations ----
    double ub[M];
#pragma unroll
    for (int v = 0; v < M; ++v) ub[v] = Gc[a * M + v];
    for (int r = p.R; r >= 1; --r) {
      for (int l = 0; l < n; ++l)
#pragma unroll
        for (int v = 0; v < M; ++v) {
          double s = 0.0;
          for (int tt = 0; tt < n; ++tt) s += p.t.P[tt][l] * at(QB, tt, v, a);
          at(RB, l, v, a) = -c * s;
        }
#pragma unroll
      for (int v = 0; v < M; ++v)
        for (int tt = 0; tt < n; ++tt) ub[v] += at(QB, tt, v, a);
      __syncthreads();
      const double* Qp = QI + (int64_t)(r - 1) * PL;
      for (int tt = 0; tt < n; ++tt) {
        double q[M], nb[M];
#pragma unroll
        for (int v = 0; v < M; ++v) {
          q[v] = Qp[(tt * M + v) * NS + a];
          nb[v] = 0.0;
        }
        static_for<0, D>([&](auto I_) {
          constexpr int I = decltype(I_)::value;
          const int ai = coord<n, I>(a), fb = face_node<n, I>(a);
          double Fi[M];
#pragma unroll
          for (int v = 0; v < M; ++v) Fi[v] = 0.0;
          for (int k = 0; k < n; ++k) {
            const int nd = pencil_node<n, I>(fb, k);
            const double dk = p.t.D[k][ai];
#pragma unroll
            for (int v = 0; v < M; ++v) Fi[v] += dk * at(RB, tt, v, nd);
          }
          PDE::template flux_adj<I>(q, Fi, nb, pb, p.g, cp);
        });
#pragma unroll
        for (int v = 0; v < M; ++v) at(QB, tt, v, a) = nb[v];
      }
      __syncthreads();
    }
#pragma unroll
    for (int v = 0; v < M; ++v)
      for (int tt = 0; tt < n; ++tt) ub[v] += at(QB, tt, v, a);
    __syncthreads();                       // every read of this cell's G is done
#pragma unroll
    for (int v = 0; v < M; ++v) p.Qbar[(cell * NS + a) * M + v] = ub[v];
    if constexpr (NPAR > 0) {
#pragma unroll
      for (int k = 0; k < NPAR; ++k) pred[k * NS + a] = pb[k];
      __syncthreads();
      if (a < NPAR && p.pbar) {
        double acc = 0.0;
        for (int j = 0; j < NS; ++j) acc += pred[a * NS + j];
        p.pbar[cell * NPAR + a] += acc;
      }
      __syncthreads();
    }
  }
}

// Reverse of one step: Qtmp <- Q; forward predictor on Qtmp (float64 traces
// of Q); k_adj_corr; k_adj_pred.  Workspace: traces, trace bars, Qtmp, slots.
template <class K>
int launch_adjoint(const LaunchArgs& a) {
  static_assert(std::is_same<typename K::Real, double>::value, "adjoint is float64");
  const int64_t qbytes = a.ncells * K::NS * K::M * 8;
  hipError_t e = hipMemcpyAsync(a.adj_qtmp, a.Qc, qbytes, hipMemcpyDeviceToDevice, a.stream);
  if (e != hipSuccess) return (int)e;
  LaunchArgs f = a;
  f.Q = a.adj_qtmp;
  int st = launch_predict<K>(f);
  if (st) return st;

  AdjCorrP<K> pc;
  pc.G = a.Qbar;
  pc.par = a.params;
  pc.dt = a.dt;
  pc.tr = reinterpret_cast<const double*>(a.traces);
  pc.tb = a.adj_tb;
  pc.pbar = a.params_bar;
  pc.ncells = a.ncells;
  for (int k = 0; k < 3; ++k) pc.nc[k] = a.nc[k];
  pc.inv_h = a.inv_h;
  for (int k = 0; k < 4; ++k) pc.g.c[k] = a.gp[k];
  for (int k = 0; k < K::n; ++k) {
    pc.LL[k] = a.tab->LL[k];
    pc.LR[k] = a.tab->LR[k];
  }
  const int64_t Gc = reduce_grid<K>(a.ncells);
  hipLaunchKernelGGL(k_adj_corr<K>, dim3((unsigned)Gc), dim3(K::CT), 0, a.stream, pc);
  e = hipGetLastError();
  if (e != hipSuccess) return (int)e;

  AdjPredP<K> pp;
  pp.Q = a.Qc;
  pp.par = a.params;
  pp.dt = a.dt;
  pp.Qbar = a.Qbar;
  pp.tb = a.adj_tb;
  pp.pbar = a.params_bar;
  pp.scratch = a.adj_slots;
  pp.slot_doubles = adj_slot_doubles<K>(a.R);
  pp.ncells = a.ncells;
  pp.inv_h = a.inv_h;
  pp.R = a.R;
  for (int k = 0; k < 4; ++k) pp.g.c[k] = a.gp[k];
  pp.t = make_ktab<K::n, double>(*a.tab);
  int64_t G = a.adj_nslots < a.ncells ? a.adj_nslots : a.ncells;
  hipLaunchKernelGGL(k_adj_pred<K>, dim3((unsigned)G), dim3(K::NS), 0, a.stream, pp);
  return (int)hipGetLastError();
}

}  // namespace adg
