// Reverse mode (discrete adjoint) of one ADER-DG step, dt held fixed.
//
// The step is Q+ = Q~ - (dt/h) sum_i (LR F*_{i,+} - LL F*_{i,-}) with
// Q~ = u + (dt/h) V(Fbar), traces from the Picard predictor q^R (Sec. 3,
// Eq. (2)-(6)).  Given G = dJ/dQ+:
//
//  k_adj_face  per face (each owned by its upper cell): the face-flux bar
//                Fb* = -(dt/h) LR^T G(left cell) + (dt/h) LL^T G(right cell),
//              its Rusanov transpose (qL, qR, fL, fR bars; the maximum speed
//              s passes its bar to the first maximal face node, left side
//              first), written as the trace bars of both cells; the
//              material bars of each side to a per (cell, face) slot.
//  k_adj_pred  per cell: recompute the Picard iterates (q^1..q^{R-1} kept
//              in a per-block scratch slot, time columns in registers,
//              pencils in LDS), map the trace bars and Kv^T G back to bars of
//              (qbar, Fbar_i), then sweep the iterations backwards:
//              rhs bar = -(dt/h) P^T qb, F_i bar = D_i^T rhs bar,
//              q^{r-1} bar = sum_i J_i(q^{r-1})^T F_i bar, u bar += sum_t q^r bar.
//  k_adj_pred_ck  linear fluxes at the default R = N + 1: the same bars by
//              the reverse of the power form (below).
//  Both predictor kernels add the face kernel's material bars of the cell.
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
  double* pf;            // per (cell, face) material bars (nullable)
  int64_t ncells;
  int nc[3];
  int brick[3];
  double inv_h;
  Gconst<double> g;
  double LL[K::n], LR[K::n];
};

// Workgroup shape of k_adj_face: one thread per (axis, face node) of the
// cell's lower faces, FCPB cells per workgroup.
template <class K>
struct AdjFace {
  static constexpr int FT = K::D * K::NF;
  static constexpr int FCPB = FT >= 256 ? 1 : 256 / FT;
  static constexpr int THREADS = FCPB * FT;
};

// Each face once: a cell takes its d lower faces (between its -e_i
// neighbour L and itself), so every face of the grid has one owner.  The
// cell's own G is staged in LDS (its pencils give LL^T G for all d faces);
// the neighbour's pencils give LR^T G.  Both sides' trace bars are written
// (the neighbour's upper face and this cell's lower face: each face slot of
// the trace-bar array has exactly one writer), and the material bars of each
// side go to a per (cell, face) slot that the predictor's reverse adds in, so
// no atomics.  Cells in the XCD-aware brick walk of the forward corrector.
template <class K>
__global__ void __launch_bounds__(AdjFace<K>::THREADS) k_adj_face(const AdjCorrP<K> p) {
  using PDE = typename K::PDE;
  constexpr int n = K::n, M = K::M, NF = K::NF, NS = K::NS, D = K::D, NPAR = K::NPAR;
  constexpr int FT = AdjFace<K>::FT, CC = AdjFace<K>::FCPB, TH = AdjFace<K>::THREADS;
  __shared__ double Gs[CC][NS * M];
  __shared__ double lamL[CC][FT], lamR[CC][FT], sbp[CC][FT];
  __shared__ double smax[CC][D], sbar[CC][D];
  __shared__ int bstar[CC][D], sstar[CC][D];
  __shared__ int64_t cid[CC];
  __shared__ double pr[NPAR > 0 ? CC * 2 * NPAR * FT : 1];
  const int lc = threadIdx.x / FT;
  const int t = threadIdx.x - lc * FT;
  const double cdt = (*p.dt) * p.inv_h;
  const int64_t groups = (p.ncells + CC - 1) / CC;
  const int64_t grp = xcd_group(groups);
  if (grp >= groups) return;                    // whole workgroup leaves together
  const int64_t gc = grp * CC + lc;
  const bool live = gc < p.ncells;
  const int64_t cell = live ? brick_cell(gc, p.nc, p.brick) : 0;
  if (t == 0) cid[lc] = live ? cell : -1;
  __syncthreads();
  for (int e = threadIdx.x; e < CC * NS * M; e += TH) {
    const int c = e / (NS * M), r = e - c * (NS * M);
    if (cid[c] >= 0) Gs[c][r] = p.G[cid[c] * NS * M + r];
  }
  __syncthreads();

  const int i = t / NF, b = t - i * NF;
  const int64_t cL = live ? neighbour<K>(cell, i, -1, p.nc) : 0;
  double qL[M], qR[M], Fb[M];
  const auto pL = PDE::template cell<double>(p.par + cL * NPAR);
  const auto pR = PDE::template cell<double>(p.par + cell * NPAR);
  if (live) {
    const double* trL = p.tr + cL * K::TRACE_ELEMS + (int64_t)(2 * i + 1) * K::NQ * NF * M + b;
    const double* trR = p.tr + cell * K::TRACE_ELEMS + (int64_t)(2 * i) * K::NQ * NF * M + b;
#pragma unroll
    for (int v = 0; v < M; ++v) {
      qL[v] = trL[v * NF];
      qR[v] = trR[v * NF];
      Fb[v] = 0.0;
    }
    static_for<0, D>([&](auto I_) {
      constexpr int I = decltype(I_)::value;
      if (i == I) {
        lamL[lc][t] = PDE::template speed<I>(qL, p.g, pL);
        lamR[lc][t] = PDE::template speed<I>(qR, p.g, pR);
        // Fb* = -(dt/h) (LR^T G_L)_b + (dt/h) (LL^T G_R)_b
        const double* GL = p.G + cL * NS * M;
#pragma unroll
        for (int k = 0; k < n; ++k) {
          const int nd = pencil_node<n, I>(b, k);
#pragma unroll
          for (int v = 0; v < M; ++v)
            Fb[v] += -cdt * p.LR[k] * GL[nd * M + v] + cdt * p.LL[k] * Gs[lc][nd * M + v];
        }
      }
    });
    double sp = 0.0;
#pragma unroll
    for (int v = 0; v < M; ++v) sp += Fb[v] * (qR[v] - qL[v]);
    sbp[lc][t] = -0.5 * sp;
  }
  __syncthreads();
  if (live && t < D) {
    // the largest speed of face t and the first node that attains it (left
    // side before right), and the bar of that speed
    double best = -1.0, acc = 0.0;
    int bs = 0, ss = 0;
    for (int bb = 0; bb < NF; ++bb) {
      const double l0 = lamL[lc][t * NF + bb], l1 = lamR[lc][t * NF + bb];
      if (l0 > best) { best = l0; bs = bb; ss = 0; }
      if (l1 > best) { best = l1; bs = bb; ss = 1; }
      acc += sbp[lc][t * NF + bb];
    }
    smax[lc][t] = best;
    bstar[lc][t] = bs;
    sstar[lc][t] = ss;
    sbar[lc][t] = acc;
  }
  __syncthreads();
  double pbs[2][NPAR > 0 ? NPAR : 1];
#pragma unroll
  for (int sd = 0; sd < 2; ++sd)
#pragma unroll
    for (int k = 0; k < (NPAR > 0 ? NPAR : 1); ++k) pbs[sd][k] = 0.0;
  if (live) {
    // side 0: this cell, the right state of the face (its lower face 2i);
    // side 1: the neighbour, the left state (its upper face 2i + 1)
#pragma unroll
    for (int sd = 0; sd < 2; ++sd) {
      double tq[M], tf[M];
      const double sgn = sd ? 0.5 : -0.5;
      const double* own = sd ? qL : qR;
#pragma unroll
      for (int v = 0; v < M; ++v) {
        tq[v] = sgn * smax[lc][i] * Fb[v];
        tf[v] = 0.5 * Fb[v];
      }
      const auto& po = sd ? pL : pR;
      const bool mine = (bstar[lc][i] == b) && (sstar[lc][i] == (sd ? 0 : 1));
      static_for<0, D>([&](auto I_) {
        constexpr int I = decltype(I_)::value;
        if (i == I) {
          if (mine) PDE::template speed_adj<I>(own, sbar[lc][i], tq, pbs[sd], p.g, po);
          if constexpr (K::NQ == 1) PDE::template flux_adj<I>(own, tf, tq, pbs[sd], p.g, po);
        }
      });
      const int64_t oc = sd ? cL : cell;
      double* out = p.tb + oc * K::TRACE_ELEMS + (int64_t)(2 * i + sd) * K::NQ * NF * M + b;
#pragma unroll
      for (int v = 0; v < M; ++v) out[v * NF] = tq[v];
      if constexpr (K::NQ == 2) {
#pragma unroll
        for (int v = 0; v < M; ++v) out[NF * M + v * NF] = tf[v];
      }
    }
  }
  if constexpr (NPAR > 0) {
#pragma unroll
    for (int sd = 0; sd < 2; ++sd)
#pragma unroll
      for (int k = 0; k < NPAR; ++k) pr[((lc * 2 + sd) * NPAR + k) * FT + t] = pbs[sd][k];
    __syncthreads();
    if (live && p.pf) {
      for (int u = t; u < 2 * D * NPAR; u += FT) {
        const int sd = u / (D * NPAR), rem = u - sd * (D * NPAR);
        const int fi = rem / NPAR, k = rem - fi * NPAR;
        double acc = 0.0;
        for (int bb = 0; bb < NF; ++bb) acc += pr[((lc * 2 + sd) * NPAR + k) * FT + fi * NF + bb];
        const int64_t oc = sd ? neighbour<K>(cell, fi, -1, p.nc) : cell;
        p.pf[(oc * 2 * D + 2 * fi + sd) * NPAR + k] = acc;
      }
    }
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
  const double* pf;      // per (cell, face) material bars of the face kernel
  double* scratch;       // per-block slots of stored Picard iterates
  int64_t slot_doubles;
  int64_t ncells;
  double inv_h;
  int R;
  Gconst<double> g;
  KTab<K::n, double> t;
};

// LDS plan of the adjoint predictor: two node-major buffers of S time slices
// per cell (published values, pencil results), S as large as 80 KiB allows.
template <class K>
struct AdjPlan {
  static constexpr int SL = K::NSP * K::MP;                 // doubles per slice
  static constexpr int pick_S() {
    for (int s = K::n; s > 1; --s)
      if (K::CPB * 2 * s * SL * 8 <= 80 * 1024) return s;
    return 1;
  }
  static constexpr int S = pick_S();
  static constexpr int NB = (K::n + S - 1) / S;
  static constexpr int CELL = 2 * S * SL;                   // doubles per cell
};

// Stored iterates q^1 .. q^{R-1} of the CPB cells of a block:
// [r-1][t][v][CPB * NS], node fastest (coalesced per thread).
template <class K>
constexpr int64_t adj_slot_doubles(int R) {
  if (K::CK && R == K::N + 1) return (int64_t)R * K::M * K::NS * K::CPB;   // k_adj_pred_ck
  const int64_t levels = R > 2 ? R - 1 : 1;
  return levels * K::n * K::M * K::NS * K::CPB;
}

// LDS index in a buffer of S time slices (the forward predictor's layout).
template <class K, int S>
__device__ __forceinline__ int alidx(int tt, int v, int pos) {
  return K::template lidx_e<S>(tt * K::NSP + K::slot(pos), v);
}

// One thread per spatial node, CPB cells per workgroup, one cell per thread
// group at a time (persistent blocks, each with its scratch slot).  The
// node thread keeps time columns in registers; spatial contractions go
// through LDS pencils exactly as in the forward predictor.
//  1. recompute q^1..q^R (first iteration on one slice), storing q^1..q^{R-1};
//  2. bars of the time averages: qbar from the q traces, Fbar_i from the flux
//     traces and the volume term (Kv^T of G), then q^R bar at every time node;
//  3. for r = R..1: u bar += sum_t q^r bar; rhs bar = -(dt/h) P^T q^r bar;
//     F_i bar = D_i^T rhs bar (pencils), q^{r-1} bar = sum_i J_i(q^{r-1})^T F_i bar
//     (r = 1: one slice with the row sums of P, q^0 = u).
template <class K>
__global__ void __launch_bounds__(K::THREADS) k_adj_pred(const AdjPredP<K> p) {
  using PDE = typename K::PDE;
  using Plan = AdjPlan<K>;
  constexpr int n = K::n, M = K::M, NS = K::NS, NF = K::NF, D = K::D, NPAR = K::NPAR;
  constexpr int CPB = K::CPB, S = Plan::S;
  __shared__ __align__(16) double smem[CPB * Plan::CELL];
  static_assert(NPAR * NS <= Plan::CELL, "material bars reuse the slice buffers");
  double* pred = smem;                         // material-bar reduction, after the sweep
  const int lc = threadIdx.x / NS;
  const int a = threadIdx.x - lc * NS;
  double* A = smem + lc * Plan::CELL;          // published slices
  double* B = A + S * Plan::SL;                // pencil results
  double* slot = p.scratch + (int64_t)blockIdx.x * p.slot_doubles;
  const int64_t LV = (int64_t)n * M * CPB * NS;
  auto it_at = [&](int r, int t, int v) -> double& {
    return slot[(r - 1) * LV + ((int64_t)(t * M + v) * CPB + lc) * NS + a];
  };
  const double c = (*p.dt) * p.inv_h;

  for (int64_t c0 = (int64_t)blockIdx.x * CPB; c0 < p.ncells; c0 += (int64_t)gridDim.x * CPB) {
    const int64_t cell = c0 + lc;
    const bool live = cell < p.ncells;
    const int64_t cs = live ? cell : 0;
    double u[M];
#pragma unroll
    for (int v = 0; v < M; ++v) u[v] = p.Q[(cs * NS + a) * M + v];
    const auto cp = PDE::template cell<double>(p.par + cs * NPAR);
    double pb[NPAR > 0 ? NPAR : 1];
#pragma unroll
    for (int k = 0; k < (NPAR > 0 ? NPAR : 1); ++k) pb[k] = 0.0;

    // Forward pencils: B <- sum_i D_i F_i(A) on ns slices.  Lanes take the
    // pencil tasks in the forward predictor's bank-conflict-free order; a
    // task is its first slot e0 (slice and pencil base), then stride sI.
    auto fwd_contract = [&](auto NS_) {
      constexpr int ns = decltype(NS_)::value;
      static_for<0, D>([&](auto I_) {
        constexpr int I = decltype(I_)::value;
        constexpr int sI = K::sstride(I);
        if (a < ns * NF) {
          const int e0 = task_e0<K, ns, I>(a);
          double out[n][M];
          pencil_dF<n, M, double>(p.t, [&](int j, double (&F)[M]) {
            double qn[M];
#pragma unroll
            for (int v = 0; v < M; ++v) qn[v] = A[K::template lidx_e<S>(e0 + j * sI, v)];
            PDE::template flux<I>(qn, F, p.g, cp);
          }, out);
          // every read of the pencil before any write: no serialised
          // read-modify-write through possibly aliasing stores
          if constexpr (I > 0) {
#pragma unroll
            for (int k = 0; k < n; ++k)
#pragma unroll
              for (int v = 0; v < M; ++v) out[k][v] += B[K::template lidx_e<S>(e0 + k * sI, v)];
          }
#pragma unroll
          for (int k = 0; k < n; ++k)
#pragma unroll
            for (int v = 0; v < M; ++v) B[K::template lidx_e<S>(e0 + k * sI, v)] = out[k][v];
        }
        __syncthreads();
      });
    };
    // Reverse pencils of axis I: B <- D_I^T A on ns slices.
    auto rev_contract = [&](auto NS_, auto I_) {
      constexpr int ns = decltype(NS_)::value, I = decltype(I_)::value;
      constexpr int sI = K::sstride(I);
      if (a < ns * NF) {
        const int e0 = task_e0<K, ns, I>(a);
        double in[n][M];
#pragma unroll
        for (int j = 0; j < n; ++j)
#pragma unroll
          for (int v = 0; v < M; ++v) in[j][v] = A[K::template lidx_e<S>(e0 + j * sI, v)];
#pragma unroll
        for (int k = 0; k < n; ++k) {
#pragma unroll
          for (int v = 0; v < M; ++v) {
            double acc = 0.0;
#pragma unroll
            for (int j = 0; j < n; ++j) acc = fma(p.t.D[j][k], in[j][v], acc);
            B[K::template lidx_e<S>(e0 + k * sI, v)] = acc;
          }
        }
      }
    };

    // ---- 1. recompute the Picard iterates ----
    double q[n][M];
#pragma unroll
    for (int v = 0; v < M; ++v) A[alidx<K, S>(0, v, a)] = u[v];
    __syncthreads();
    fwd_contract(std::integral_constant<int, 1>{});
#pragma unroll
    for (int v = 0; v < M; ++v) {
      const double rv = B[alidx<K, S>(0, v, a)];
#pragma unroll
      for (int t = 0; t < n; ++t) q[t][v] = u[v] - c * (p.t.Ps[t] * rv);
    }
    for (int r = 2; r <= p.R; ++r) {
#pragma unroll
      for (int t = 0; t < n; ++t)
#pragma unroll
        for (int v = 0; v < M; ++v) it_at(r - 1, t, v) = q[t][v];
      double acc[n][M];
#pragma unroll
      for (int t = 0; t < n; ++t)
#pragma unroll
        for (int v = 0; v < M; ++v) acc[t][v] = 0.0;
      static_for<0, Plan::NB>([&](auto B_) {
        constexpr int t0 = decltype(B_)::value * S;
        constexpr int ns = (n - t0) < S ? (n - t0) : S;
        __syncthreads();                       // previous readers of A and B are done
#pragma unroll
        for (int tt = 0; tt < ns; ++tt)
#pragma unroll
          for (int v = 0; v < M; ++v) A[alidx<K, S>(tt, v, a)] = q[t0 + tt][v];
        __syncthreads();
        fwd_contract(std::integral_constant<int, ns>{});
#pragma unroll
        for (int tt = 0; tt < ns; ++tt)
#pragma unroll
          for (int v = 0; v < M; ++v) {
            const double rv = B[alidx<K, S>(tt, v, a)];
#pragma unroll
            for (int t = 0; t < n; ++t) acc[t][v] = fma(p.t.P[t][t0 + tt], rv, acc[t][v]);
          }
      });
#pragma unroll
      for (int t = 0; t < n; ++t)
#pragma unroll
        for (int v = 0; v < M; ++v) q[t][v] = u[v] - c * acc[t][v];
    }

    // ---- 2. bars of qbar and Fbar_i at this node, then q^R bar ----
    const double* TB = p.tb + cs * K::TRACE_ELEMS;
    const double* Gc = p.Qbar + cs * NS * M;
    double qb[n][M];
    {
      double qbb[M], Fbb[D][M];
#pragma unroll
      for (int v = 0; v < M; ++v) qbb[v] = 0.0;
      static_for<0, D>([&](auto I_) {
        constexpr int I = decltype(I_)::value;
        const int ai = coord<n, I>(a), fb = face_node<n, I>(a);
        const double* tl = TB + (int64_t)(2 * I) * K::NQ * NF * M + fb;
        const double* trr = TB + (int64_t)(2 * I + 1) * K::NQ * NF * M + fb;
#pragma unroll
        for (int v = 0; v < M; ++v) {
          qbb[v] += p.t.FL[ai] * tl[v * NF] + p.t.FR[ai] * trr[v * NF];
          Fbb[I][v] = (K::NQ == 2) ? p.t.FL[ai] * tl[NF * M + v * NF] + p.t.FR[ai] * trr[NF * M + v * NF] : 0.0;
        }
#pragma unroll
        for (int k = 0; k < n; ++k) {
          const int nd = pencil_node<n, I>(fb, k);
          const double kv = c * p.t.Kv[k][ai];
#pragma unroll
          for (int v = 0; v < M; ++v) Fbb[I][v] += kv * Gc[nd * M + v];
        }
      });
#pragma unroll
      for (int t = 0; t < n; ++t) {
        const double wt = p.t.w[t];
#pragma unroll
        for (int v = 0; v < M; ++v) qb[t][v] = wt * qbb[v];
        static_for<0, D>([&](auto I_) {
          constexpr int I = decltype(I_)::value;
          double fw[M];
#pragma unroll
          for (int v = 0; v < M; ++v) fw[v] = wt * Fbb[I][v];
          PDE::template flux_adj<I>(q[t], fw, qb[t], pb, p.g, cp);
        });
      }
    }
    double ub[M];
#pragma unroll
    for (int v = 0; v < M; ++v) ub[v] = Gc[a * M + v];

    // ---- 3. reverse sweep over the Picard iterations ----
    for (int r = p.R; r >= 2; --r) {
      double rb[n][M], nb[n][M];
#pragma unroll
      for (int v = 0; v < M; ++v) {
#pragma unroll
        for (int t = 0; t < n; ++t) ub[v] += qb[t][v];
#pragma unroll
        for (int l = 0; l < n; ++l) {
          double s = 0.0;
#pragma unroll
          for (int t = 0; t < n; ++t) s = fma(p.t.P[t][l], qb[t][v], s);
          rb[l][v] = -c * s;
        }
      }
#pragma unroll
      for (int l = 0; l < n; ++l)
#pragma unroll
        for (int v = 0; v < M; ++v) nb[l][v] = 0.0;
      static_for<0, Plan::NB>([&](auto B_) {
        constexpr int l0 = decltype(B_)::value * S;
        constexpr int ns = (n - l0) < S ? (n - l0) : S;
        double qp[ns][M];
#pragma unroll
        for (int tt = 0; tt < ns; ++tt)
#pragma unroll
          for (int v = 0; v < M; ++v) qp[tt][v] = it_at(r - 1, l0 + tt, v);
        __syncthreads();                       // previous readers of A and B are done
#pragma unroll
        for (int tt = 0; tt < ns; ++tt)
#pragma unroll
          for (int v = 0; v < M; ++v) A[alidx<K, S>(tt, v, a)] = rb[l0 + tt][v];
        __syncthreads();
        static_for<0, D>([&](auto I_) {
          constexpr int I = decltype(I_)::value;
          if constexpr (I > 0) __syncthreads();   // B read by every node below
          rev_contract(std::integral_constant<int, ns>{}, I_);
          __syncthreads();
#pragma unroll
          for (int tt = 0; tt < ns; ++tt) {
            double fb[M];
#pragma unroll
            for (int v = 0; v < M; ++v) fb[v] = B[alidx<K, S>(tt, v, a)];
            PDE::template flux_adj<I>(qp[tt], fb, nb[l0 + tt], pb, p.g, cp);
          }
        });
      });
#pragma unroll
      for (int t = 0; t < n; ++t)
#pragma unroll
        for (int v = 0; v < M; ++v) qb[t][v] = nb[t][v];
    }
    // r = 1: q^1 = u - (dt/h) Ps rhs(u), one slice
    {
      double rb0[M];
#pragma unroll
      for (int v = 0; v < M; ++v) {
        double s = 0.0;
#pragma unroll
        for (int t = 0; t < n; ++t) {
          ub[v] += qb[t][v];
          s = fma(p.t.Ps[t], qb[t][v], s);
        }
        rb0[v] = -c * s;
      }
      __syncthreads();
#pragma unroll
      for (int v = 0; v < M; ++v) A[alidx<K, S>(0, v, a)] = rb0[v];
      __syncthreads();
      static_for<0, D>([&](auto I_) {
        constexpr int I = decltype(I_)::value;
        if constexpr (I > 0) __syncthreads();
        rev_contract(std::integral_constant<int, 1>{}, I_);
        __syncthreads();
        double fb[M];
#pragma unroll
        for (int v = 0; v < M; ++v) fb[v] = B[alidx<K, S>(0, v, a)];
        PDE::template flux_adj<I>(u, fb, ub, pb, p.g, cp);
      });
    }
    __syncthreads();                       // every read of this cell's G is done
    if (live) {
#pragma unroll
      for (int v = 0; v < M; ++v) p.Qbar[(cell * NS + a) * M + v] = ub[v];
    }
    if constexpr (NPAR > 0) {
#pragma unroll
      for (int k = 0; k < NPAR; ++k) pred[(lc * NPAR + k) * NS + a] = pb[k];
      __syncthreads();
      if (a < NPAR && live && p.pbar) {
        double acc = 0.0;
        for (int j = 0; j < NS; ++j) acc += pred[(lc * NPAR + a) * NS + j];
        for (int f = 0; f < 2 * D; ++f) acc += p.pf[(cell * 2 * D + f) * NPAR + a];
        p.pbar[cell * NPAR + a] += acc;
      }
    }
    __syncthreads();                       // LDS and pred reused by the next cell
  }
}

// Long float64 time columns (the forward predictor's gather form, n >= 7,
// nonlinear flux): the same reverse sweep as k_adj_pred with every spatial
// contraction done by gathers at the node threads instead of pencil tasks,
// slice by slice, with two LDS buffers in turn (one barrier per slice):
//  1. recompute q^1..q^R (q^1..q^{R-1} to the block's slot, q^R kept);
//  2. bars of qbar and Fbar_i from the trace bars and Kv^T G (tables in LDS);
//  3. for r = R..2: u bar += sum_t q^r bar; per slice l: rhs bar_l =
//     -(dt/h) sum_t P[t][l] q^r bar_t is published, each node gathers
//     F_i bar = D_i^T rhs bar_l along its d pencils and adds
//     J_i(q^{r-1}_l)^T F_i bar to q^{r-1} bar_l;
//  4. r = 1 on one slice with the row sums of P, Jacobians at u.
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

template <class K>
struct AdjGather {
  static constexpr int PL = K::D * K::NSP * K::MP;           // doubles of one flux-plane set
  static constexpr int DR = K::n + 1;                        // padded table rows
  static constexpr int TAB = 3 * K::n * DR + 2 * K::n;       // D, Kv, P, FL, FR
  static constexpr int CELL = 2 * PL + TAB;
};

template <class K>
__global__ void __launch_bounds__(K::NODE_THREADS) k_adj_pred_g(const AdjPredP<K> p) {
  using PDE = typename K::PDE;
  using Gp = AdjGather<K>;
  constexpr int n = K::n, M = K::M, NS = K::NS, NF = K::NF, D = K::D, NPAR = K::NPAR;
  constexpr int NSP = K::NSP, PL = Gp::PL, DR = Gp::DR;
  static_assert(K::CPB == 1, "one cell per workgroup");
  static_assert(NPAR * NS <= 2 * PL, "material bars reuse the flux planes");
  __shared__ __align__(16) double smem[Gp::CELL];
  double* Fp = smem;                                   // two flux-plane sets
  double* sD = smem + 2 * PL;                          // D[k][j] at k * DR + j
  double* sKv = sD + n * DR;
  double* sP = sKv + n * DR;                           // P[t][l] at t * DR + l
  double* sFL = sP + n * DR;
  double* sFR = sFL + n;
  const int a = threadIdx.x;
  // tables by static indices (a lane-dependent index into the kernel
  // argument would copy the whole argument block to scratch memory); P too:
  // read in the loops from LDS, its n^2 values are not held in registers
  if (a == 0) {
#pragma unroll
    for (int i = 0; i < n * n; ++i) {
      sD[(i / n) * DR + i % n] = p.t.D[i / n][i % n];
      sKv[(i / n) * DR + i % n] = p.t.Kv[i / n][i % n];
      sP[(i / n) * DR + i % n] = p.t.P[i / n][i % n];
    }
#pragma unroll
    for (int i = 0; i < n; ++i) {
      sFL[i] = p.t.FL[i];
      sFR[i] = p.t.FR[i];
    }
  }
  // The block's slot of stored iterates through buffer instructions: a
  // scalar resource and offset per (r, t, v) and one lane offset register,
  // where 64-bit lane addresses would hold a register pair per access.
  double* slot = p.scratch + (int64_t)blockIdx.x * p.slot_doubles;
  const __amdgpu_buffer_rsrc_t srs =
      __builtin_amdgcn_make_buffer_rsrc(slot, (short)0, (int)(p.slot_doubles * 8), 0x00020000);
  const int LVB = n * M * NS * 8;                      // bytes of one iterate
  const int lane_off = a * 8;
  auto it_st = [&](int r, int t, int v, double x) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, x), srs, lane_off,
                                          (r - 1) * LVB + (t * M + v) * NS * 8, 0);
  };
  auto it_ld = [&](int r, int t, int v) -> double {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(srs, lane_off,
                                                                           (r - 1) * LVB + (t * M + v) * NS * 8, 0));
  };
  const double c = (*p.dt) * p.inv_h;
  int g = 0;                                           // gathers so far: buffer g % 2

  for (int64_t cell = blockIdx.x; cell < p.ncells; cell += gridDim.x) {
    double u[M];
#pragma unroll
    for (int v = 0; v < M; ++v) u[v] = p.Q[(cell * NS + a) * M + v];
    const auto cp = PDE::template cell<double>(p.par + cell * NPAR);
    double pb[NPAR > 0 ? NPAR : 1];
#pragma unroll
    for (int k = 0; k < (NPAR > 0 ? NPAR : 1); ++k) pb[k] = 0.0;

    // rv = sum_i D_i F_i(x) at this node (forward gather)
    auto gather_f = [&](const double (&x)[M], double (&rv)[M]) {
      double* Fs = Fp + (g & 1) * PL;
      ++g;
      double w[M];
      PDE::pub(x, w, p.g);
      static_for<0, D>([&](auto I_) {
        constexpr int I = decltype(I_)::value;
        double F[M];
        PDE::template flux_pub<I>(w, F, p.g, cp);
#pragma unroll
        for (int v = 0; v < M; ++v) Fs[K::template lidx_e<D>(I * NSP + K::slot(a), v)] = F[v];
      });
      __syncthreads();
#pragma unroll
      for (int v = 0; v < M; ++v) rv[v] = 0.0;
      static_for<0, D>([&](auto I_) {
        constexpr int I = decltype(I_)::value;
        constexpr int sI = K::sstride(I);
        const int ai = coord<n, I>(a);
        const int e0 = I * NSP + K::slot(a) - ai * sI;
#pragma unroll
        for (int j = 0; j < n; ++j) {
          const double dj = sD[ai * DR + j];
#pragma unroll
          for (int v = 0; v < M; ++v) rv[v] = fma(dj, Fs[K::template lidx_e<D>(e0 + j * sI, v)], rv[v]);
        }
      });
    };
    // out += sum_i J_i(z)^T (D_i^T y) at this node (reverse gather of y)
    auto gather_r = [&](const double (&y)[M], const double (&z)[M], double (&out)[M]) {
      double* Fs = Fp + (g & 1) * PL;
      ++g;
#pragma unroll
      for (int v = 0; v < M; ++v) Fs[K::template lidx_e<D>(K::slot(a), v)] = y[v];
      __syncthreads();
      static_for<0, D>([&](auto I_) {
        constexpr int I = decltype(I_)::value;
        constexpr int sI = K::sstride(I);
        const int ai = coord<n, I>(a);
        const int e0 = K::slot(a) - ai * sI;
        double fb[M];
#pragma unroll
        for (int v = 0; v < M; ++v) fb[v] = 0.0;
#pragma unroll
        for (int k = 0; k < n; ++k) {
          const double dk = sD[k * DR + ai];
#pragma unroll
          for (int v = 0; v < M; ++v) fb[v] = fma(dk, Fs[K::template lidx_e<D>(e0 + k * sI, v)], fb[v]);
        }
        PDE::template flux_adj<I>(z, fb, out, pb, p.g, cp);
      });
    };

    // ---- 1. recompute the Picard iterates ----
    double q[n][M];
    {
      double rv[M];
      gather_f(u, rv);
#pragma unroll
      for (int v = 0; v < M; ++v)
#pragma unroll
        for (int t = 0; t < n; ++t) q[t][v] = u[v] - c * (p.t.Ps[t] * rv[v]);
    }
    for (int r = 2; r <= p.R; ++r) {
      double acc[n][M];
#pragma unroll
      for (int t = 0; t < n; ++t)
#pragma unroll
        for (int v = 0; v < M; ++v) {
          it_st(r - 1, t, v, q[t][v]);
          acc[t][v] = 0.0;
        }
      static_for<0, n>([&](auto T_) {
        constexpr int tt = decltype(T_)::value;
        double rv[M];
        gather_f(q[tt], rv);
#pragma unroll
        for (int t = 0; t < n; ++t)
#pragma unroll
          for (int v = 0; v < M; ++v) acc[t][v] = fma(sP[t * DR + tt], rv[v], acc[t][v]);
      });
#pragma unroll
      for (int t = 0; t < n; ++t)
#pragma unroll
        for (int v = 0; v < M; ++v) q[t][v] = u[v] - c * acc[t][v];
    }

    // ---- 2. bars of qbar and Fbar_i at this node, then q^R bar ----
    const double* TB = p.tb + cell * K::TRACE_ELEMS;
    const double* Gc = p.Qbar + cell * NS * M;
    double qb[n][M];
    {
      double qbb[M], Fbb[D][M];
#pragma unroll
      for (int v = 0; v < M; ++v) qbb[v] = 0.0;
      static_for<0, D>([&](auto I_) {
        constexpr int I = decltype(I_)::value;
        __builtin_amdgcn_sched_barrier(0);               // one axis's loads in flight
        const int ai = coord<n, I>(a), fb = face_node<n, I>(a);
        const double* tl = TB + (int64_t)(2 * I) * K::NQ * NF * M + fb;
        const double* trr = TB + (int64_t)(2 * I + 1) * K::NQ * NF * M + fb;
        const double fl = sFL[ai], fr = sFR[ai];
#pragma unroll
        for (int v = 0; v < M; ++v) {
          qbb[v] += fl * tl[v * NF] + fr * trr[v * NF];
          Fbb[I][v] = (K::NQ == 2) ? fl * tl[NF * M + v * NF] + fr * trr[NF * M + v * NF] : 0.0;
        }
#pragma unroll
        for (int k = 0; k < n; ++k) {
          const int nd = pencil_node<n, I>(fb, k);
          const double kv = c * sKv[k * DR + ai];
#pragma unroll
          for (int v = 0; v < M; ++v) Fbb[I][v] += kv * Gc[nd * M + v];
        }
      });
#pragma unroll
      for (int t = 0; t < n; ++t) {
        __builtin_amdgcn_sched_barrier(0);               // slices one at a time
        const double wt = p.t.w[t];
#pragma unroll
        for (int v = 0; v < M; ++v) qb[t][v] = wt * qbb[v];
        static_for<0, D>([&](auto I_) {
          constexpr int I = decltype(I_)::value;
          double fw[M];
#pragma unroll
          for (int v = 0; v < M; ++v) fw[v] = wt * Fbb[I][v];
          PDE::template flux_adj<I>(q[t], fw, qb[t], pb, p.g, cp);
        });
      }
    }
    double ub[M];
#pragma unroll
    for (int v = 0; v < M; ++v) ub[v] = Gc[a * M + v];

    // ---- 3. reverse sweep over the Picard iterations ----
    // (all rhs bars first: then the q^r bars are dead, and the rhs bars of
    // the slices still to come and the q^{r-1} bars of the slices done
    // together hold n m values)
    for (int r = p.R; r >= 2; --r) {
      double rb[n][M];
#pragma unroll
      for (int v = 0; v < M; ++v) {
#pragma unroll
        for (int t = 0; t < n; ++t) ub[v] += qb[t][v];
#pragma unroll
        for (int l = 0; l < n; ++l) {
          double s = 0.0;
#pragma unroll
          for (int t = 0; t < n; ++t) s = fma(sP[t * DR + l], qb[t][v], s);
          rb[l][v] = -c * s;
        }
      }
      // the stored iterate of slice l + 1 is loaded before the barrier of
      // slice l, so its latency overlaps that slice's gather
      double zc[M];
#pragma unroll
      for (int v = 0; v < M; ++v) zc[v] = it_ld(r - 1, 0, v);
      static_for<0, n>([&](auto L_) {
        constexpr int l = decltype(L_)::value;
        double zn[M];
#pragma unroll
        for (int v = 0; v < M; ++v) {
          zn[v] = (l + 1 < n) ? it_ld(r - 1, l + 1 < n ? l + 1 : l, v) : 0.0;
          qb[l][v] = 0.0;
        }
        gather_r(rb[l], zc, qb[l]);
#pragma unroll
        for (int v = 0; v < M; ++v) zc[v] = zn[v];
      });
    }
    // r = 1: q^1 = u - (dt/h) Ps rhs(u), one slice
    {
      double rb0[M];
#pragma unroll
      for (int v = 0; v < M; ++v) {
        double s = 0.0;
#pragma unroll
        for (int t = 0; t < n; ++t) {
          ub[v] += qb[t][v];
          s = fma(p.t.Ps[t], qb[t][v], s);
        }
        rb0[v] = -c * s;
      }
      gather_r(rb0, u, ub);
    }
    __syncthreads();                       // every read of this cell's G and LDS is done
#pragma unroll
    for (int v = 0; v < M; ++v) p.Qbar[(cell * NS + a) * M + v] = ub[v];
    if constexpr (NPAR > 0) {
      double* pred = smem;
#pragma unroll
      for (int k = 0; k < NPAR; ++k) pred[k * NS + a] = pb[k];
      __syncthreads();
      if (a < NPAR && p.pbar) {
        double acc = 0.0;
        for (int j = 0; j < NS; ++j) acc += pred[a * NS + j];
        for (int f = 0; f < 2 * D; ++f) acc += p.pf[(cell * 2 * D + f) * NPAR + a];
        p.pbar[cell * NPAR + a] += acc;
      }
      __syncthreads();
    }
  }
}

// Linear fluxes (the power form of the forward predictor, see pred_cell): the
// time average is qbar = z_0 of the Horner recursion z_R = a_R u,
// z_k = a_k u + L z_{k+1}, a_k = (-dt/h)^k w.T_k (T_0 = 1, T_k = P^{k-1} Ps),
// L = sum_i D_i F_i.  Per cell:
//  1. forward Horner: R gathers of L; z_1..z_R are kept when material bars
//     are wanted (they are the states of the bilinear material terms; the
//     Jacobians themselves do not depend on the state), in LDS beside the
//     gather planes when they fit, else in the block's scratch slot;
//  2. bars of qbar and Fbar_i = F_i(qbar) from the trace bars and Kv^T G, as
//     in k_adj_pred; zbar_0 = qbar bar + sum_i J_i^T Fbar_i bar;
//  3. reverse Horner: u bar += a_k zbar_k, zbar_{k+1} = L^T zbar_k,
//     params bar += (d(L z_{k+1})/d params)^T zbar_k; u bar += a_R zbar_R.
// L^T y = sum_i J_i^T (D_i^T y), gathered along the d pencils through each
// node.  No Picard iterates and no time slices: 2R gathers of one field
// against R sweeps over n slices.  Used for R = N + 1 (the default).
template <class K>
// (At least two waves per SIMD: the large-m instantiations then spill a
// few registers instead of running one wave per SIMD.)
__global__ void __launch_bounds__(K::NODE_THREADS) __attribute__((amdgpu_waves_per_eu(2))) k_adj_pred_ck(const AdjPredP<K> p) {
  using PDE = typename K::PDE;
  constexpr int n = K::n, M = K::M, NS = K::NS, NF = K::NF, D = K::D, NPAR = K::NPAR;
  constexpr int CPB = K::CPB, NSP = K::NSP, RR = K::N + 1;
  // the gathers use the first of D plane slots: the one-plane layout (a
  // third of the LDS, six workgroups per CU instead of five for C4)
  // measured slower
  constexpr int CELLD = D * NSP * K::MP;                  // doubles of LDS per cell
  // z_1..z_R of the material terms in LDS when they fit beside the gather
  // planes, else in the block's scratch slot
  constexpr int ZD = RR * M * NS * CPB;
  constexpr bool ZLDS = NPAR > 0 && (CPB * CELLD + ZD) * 8 <= 48 * 1024;
  static_assert(NPAR * NS <= CELLD, "material bars reuse the gather planes");
  __shared__ __align__(16) double smem[CPB * CELLD + (ZLDS ? ZD : 0)];
  __shared__ double s_al[RR + 1];
  __shared__ double s_D[n][n];           // in LDS: read inside the loops, not held live
  double* pred = smem;
  const int lc = threadIdx.x / NS;
  const int a = threadIdx.x - lc * NS;
  double* Fs = smem + lc * CELLD;                          // [var][node] plane (slots of plane 0)
  const double c = (*p.dt) * p.inv_h;
  for (int i = threadIdx.x; i < n * n; i += K::NODE_THREADS) s_D[i / n][i % n] = p.t.D[i / n][i % n];
  if (threadIdx.x == 0) {
    // a_k = (-dt/h)^k w.T_k for k = 0..R (R = N + 1), the forward's table
    double ck = 1.0;
    s_al[0] = 1.0;
#pragma unroll
    for (int k = 1; k <= RR; ++k) {
      ck *= -c;
      s_al[k] = ck * p.t.beta[k - 1];
    }
  }
  __syncthreads();
  // z_k of this thread's node in the block's slot: [k-1][var][thread]
  const bool keep = NPAR > 0 && p.pbar != nullptr;
  double* zs = (ZLDS ? smem + CPB * CELLD : p.scratch + (int64_t)blockIdx.x * p.slot_doubles) + threadIdx.x;
  auto zat = [&](int k, int v) -> double& { return zs[((int64_t)(k - 1) * M + v) * (CPB * NS)]; };

  for (int64_t c0 = (int64_t)blockIdx.x * CPB; c0 < p.ncells; c0 += (int64_t)gridDim.x * CPB) {
    const int64_t cell = c0 + lc;
    const bool live = cell < p.ncells;
    const int64_t cs = live ? cell : 0;
    double u[M];
#pragma unroll
    for (int v = 0; v < M; ++v) u[v] = p.Q[(cs * NS + a) * M + v];
    const auto cp = PDE::template cell<double>(p.par + cs * NPAR);
    double pb[NPAR > 0 ? NPAR : 1];
#pragma unroll
    for (int k = 0; k < (NPAR > 0 ? NPAR : 1); ++k) pb[k] = 0.0;

    // z <- a_k u + L z (every node thread gives its z).  F_i(z) = A_i z with
    // the cell's constant material, so L z = sum_i A_i (D_i z): one plane of
    // z, gathered along the d pencils, the flux of each axis at the node.
    double z[M];
    auto horner = [&](int k) {
      __syncthreads();                                    // earlier readers of Fs done
#pragma unroll
      for (int v = 0; v < M; ++v) Fs[K::template lidx_e<D>(K::slot(a), v)] = z[v];
      __syncthreads();
      const double ak = s_al[k];
#pragma unroll
      for (int v = 0; v < M; ++v) z[v] = ak * u[v];
      static_for<0, D>([&](auto I_) {
        constexpr int I = decltype(I_)::value;
        constexpr int sI = K::sstride(I);
        const int ai = coord<n, I>(a);
        const int e0 = K::slot(a) - ai * sI;
        double dr[n], g[M], F[M];
#pragma unroll
        for (int j = 0; j < n; ++j) dr[j] = s_D[ai][j];
#pragma unroll
        for (int v = 0; v < M; ++v) {
          g[v] = 0.0;
#pragma unroll
          for (int j = 0; j < n; ++j) g[v] = fma(dr[j], Fs[K::template lidx_e<D>(e0 + j * sI, v)], g[v]);
        }
        PDE::template flux<I>(g, F, p.g, cp);
#pragma unroll
        for (int v = 0; v < M; ++v) z[v] += F[v];
      });
    };
    // zb <- L^T zb with the state zk of the material terms; u bar += a_k zb first
    double zb[M], ub[M];
    auto horner_rev = [&](int k, const double (&zk)[M]) {
      const double ak = s_al[k];
#pragma unroll
      for (int v = 0; v < M; ++v) ub[v] = fma(ak, zb[v], ub[v]);
      __syncthreads();
#pragma unroll
      for (int v = 0; v < M; ++v) Fs[K::template lidx_e<D>(K::slot(a), v)] = zb[v];
      __syncthreads();
      double nz[M];
#pragma unroll
      for (int v = 0; v < M; ++v) nz[v] = 0.0;
      static_for<0, D>([&](auto I_) {
        constexpr int I = decltype(I_)::value;
        constexpr int sI = K::sstride(I);
        __builtin_amdgcn_sched_barrier(0);
        const int ai = coord<n, I>(a);
        const int e0 = K::slot(a) - ai * sI;
        double g[M];
#pragma unroll
        for (int v = 0; v < M; ++v) g[v] = 0.0;
#pragma unroll
        for (int j = 0; j < n; ++j) {
          const double dj = s_D[j][ai];
#pragma unroll
          for (int v = 0; v < M; ++v) g[v] = fma(dj, Fs[K::template lidx_e<D>(e0 + j * sI, v)], g[v]);
        }
        PDE::template flux_adj<I>(zk, g, nz, pb, p.g, cp);
      });
#pragma unroll
      for (int v = 0; v < M; ++v) zb[v] = nz[v];
    };

    // ---- 1. forward Horner: z_R = a_R u, then down to z_0 = qbar ----
#pragma unroll
    for (int v = 0; v < M; ++v) z[v] = s_al[RR] * u[v];
#pragma unroll 1
    for (int k = RR - 1; k >= 0; --k) {
      if (keep) {
#pragma unroll
        for (int v = 0; v < M; ++v) zat(k + 1, v) = z[v];
      }
      horner(k);
    }

    // ---- 2. bars of qbar = z_0 and Fbar_i at this node ----
    const double* TB = p.tb + cs * K::TRACE_ELEMS;
    const double* Gc = p.Qbar + cs * NS * M;
#pragma unroll
    for (int v = 0; v < M; ++v) zb[v] = 0.0;
    static_for<0, D>([&](auto I_) {
      constexpr int I = decltype(I_)::value;
      __builtin_amdgcn_sched_barrier(0);                 // one axis's loads live at a time
      const int ai = coord<n, I>(a), fb = face_node<n, I>(a);
      const double* tl = TB + (int64_t)(2 * I) * K::NQ * NF * M + fb;
      const double* trr = TB + (int64_t)(2 * I + 1) * K::NQ * NF * M + fb;
      double Fbb[M];
#pragma unroll
      for (int v = 0; v < M; ++v) {
        zb[v] += p.t.FL[ai] * tl[v * NF] + p.t.FR[ai] * trr[v * NF];
        Fbb[v] = 0.0;
      }
#pragma unroll
      for (int k = 0; k < n; ++k) {
        const int nd = pencil_node<n, I>(fb, k);
        const double kv = c * p.t.Kv[k][ai];
#pragma unroll
        for (int v = 0; v < M; ++v) Fbb[v] += kv * Gc[nd * M + v];
      }
      PDE::template flux_adj<I>(z, Fbb, zb, pb, p.g, cp);
    });
#pragma unroll
    for (int v = 0; v < M; ++v) ub[v] = Gc[a * M + v];

    // ---- 3. reverse Horner ----
#pragma unroll 1
    for (int k = 0; k < RR; ++k) {
      double zk[M];
#pragma unroll
      for (int v = 0; v < M; ++v) zk[v] = keep ? zat(k + 1, v) : 0.0;   // only material terms read it
      horner_rev(k, zk);
    }
    {
      const double aR = s_al[RR];
#pragma unroll
      for (int v = 0; v < M; ++v) ub[v] = fma(aR, zb[v], ub[v]);
    }
    __syncthreads();                       // every read of this cell's G and Fs is done
    if (live) {
#pragma unroll
      for (int v = 0; v < M; ++v) p.Qbar[(cell * NS + a) * M + v] = ub[v];
    }
    if constexpr (NPAR > 0) {
#pragma unroll
      for (int k = 0; k < NPAR; ++k) pred[(lc * NPAR + k) * NS + a] = pb[k];
      __syncthreads();
      if (a < NPAR && live && p.pbar) {
        double acc = 0.0;
        for (int j = 0; j < NS; ++j) acc += pred[(lc * NPAR + a) * NS + j];
        for (int f = 0; f < 2 * D; ++f) acc += p.pf[(cell * 2 * D + f) * NPAR + a];
        p.pbar[cell * NPAR + a] += acc;
      }
    }
    __syncthreads();                       // LDS reused by the next cell
  }
}

// Reverse of one step: forward predictor of Q for its float64 traces (no Q~
// written, Q untouched); k_adj_face; k_adj_pred or k_adj_pred_ck.  Workspace:
// traces, trace bars, slots, per (cell, face) material bars.
template <class K>
int launch_adjoint(const LaunchArgs& a) {
  static_assert(std::is_same<typename K::Real, double>::value, "adjoint is float64");
  // forward traces of Q (the hull only: Q is read, nothing else written)
  LaunchArgs f = a;
  f.qin = a.Qc;
  f.traces_only = true;
  int st = launch_predict<K>(f);
  if (st) return st;
  hipError_t e;

  AdjCorrP<K> pc;
  pc.G = a.Qbar;
  pc.par = a.params;
  pc.dt = a.dt;
  pc.tr = reinterpret_cast<const double*>(a.traces);
  pc.tb = a.adj_tb;
  pc.pf = a.params_bar ? a.adj_pf : nullptr;
  pc.ncells = a.ncells;
  for (int k = 0; k < 3; ++k) pc.nc[k] = a.nc[k];
  pc.inv_h = a.inv_h;
  for (int k = 0; k < 4; ++k) pc.g.c[k] = a.gp[k];
  for (int k = 0; k < K::n; ++k) {
    pc.LL[k] = a.tab->LL[k];
    pc.LR[k] = a.tab->LR[k];
  }
  for (int k = 0; k < 3; ++k) pc.brick[k] = a.brick[k];
  const int64_t groups = (a.ncells + AdjFace<K>::FCPB - 1) / AdjFace<K>::FCPB;
  const int64_t Gc = 8 * ((groups + 7) / 8);
  hipLaunchKernelGGL(k_adj_face<K>, dim3((unsigned)Gc), dim3(AdjFace<K>::THREADS), 0, a.stream, pc);
  e = hipGetLastError();
  if (e != hipSuccess) return (int)e;

  AdjPredP<K> pp;
  pp.Q = a.Qc;
  pp.par = a.params;
  pp.dt = a.dt;
  pp.Qbar = a.Qbar;
  pp.tb = a.adj_tb;
  pp.pbar = a.params_bar;
  pp.pf = a.adj_pf;
  pp.scratch = a.adj_slots;
  pp.slot_doubles = adj_slot_doubles<K>(a.R);
  pp.ncells = a.ncells;
  pp.inv_h = a.inv_h;
  pp.R = a.R;
  for (int k = 0; k < 4; ++k) pp.g.c[k] = a.gp[k];
  pp.t = make_ktab<K::n, double>(*a.tab);
  if constexpr (K::CK) {
    if (a.R == K::N + 1) {
      // linear flux, default R: the reverse of the power form
      static int resident_ck = 0;
      if (resident_ck == 0) {
        int dev = 0, cus = 0, per_cu = 0;
        e = hipGetDevice(&dev);
        if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e == hipSuccess)
          e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_adj_pred_ck<K>, K::NODE_THREADS, 0);
        if (e != hipSuccess) return (int)e;
        resident_ck = cus * (per_cu > 0 ? per_cu : 1);
      }
      int64_t G = (a.ncells + K::CPB - 1) / K::CPB;
      if (G > a.adj_nslots) G = a.adj_nslots;
      if (G > resident_ck) G = resident_ck;
      hipLaunchKernelGGL(k_adj_pred_ck<K>, dim3((unsigned)G), dim3(K::NODE_THREADS), 0, a.stream, pp);
      return (int)hipGetLastError();
    }
  }
  if constexpr (K::GATHER) {
    // long float64 columns: the gather form (one cell per workgroup)
    static int resident_g = 0;
    if (resident_g == 0) {
      int dev = 0, cus = 0, per_cu = 0;
      e = hipGetDevice(&dev);
      if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
      if (e == hipSuccess)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_adj_pred_g<K>, K::NODE_THREADS, 0);
      if (e != hipSuccess) return (int)e;
      resident_g = cus * (per_cu > 0 ? per_cu : 1);
    }
    int64_t G = a.ncells;
    if (G > a.adj_nslots) G = a.adj_nslots;
    if (G > resident_g) G = resident_g;
    hipLaunchKernelGGL(k_adj_pred_g<K>, dim3((unsigned)G), dim3(K::NODE_THREADS), 0, a.stream, pp);
    return (int)hipGetLastError();
  }
  // Persistent blocks: no more than fit on the device at once, so every
  // block starts together and walks the same number of cells.
  static int resident = 0;
  if (resident == 0) {
    int dev = 0, cus = 0, per_cu = 0;
    e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess)
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_adj_pred<K>, K::THREADS, 0);
    if (e != hipSuccess) return (int)e;
    resident = cus * (per_cu > 0 ? per_cu : 1);
  }
  int64_t G = (a.ncells + K::CPB - 1) / K::CPB;
  if (G > a.adj_nslots) G = a.adj_nslots;
  if (G > resident) G = resident;
  hipLaunchKernelGGL(k_adj_pred<K>, dim3((unsigned)G), dim3(K::THREADS), 0, a.stream, pp);
  return (int)hipGetLastError();
}

}  // namespace adg
