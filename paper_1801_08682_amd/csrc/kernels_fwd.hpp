// Forward kernels of one ADER-DG step for gfx950.
//
//  k_pred  predict + extrapolate + integrateVolume     (Sec. 3 step 1, Eq. (3);
//          Table 1; Sec. 5 Technique 1: volume integral right after predict)
//  k_corr  solveRiemann (Rusanov, Eq. (4)) + integrateFace + update +
//          calcTimeStep (Sec. 3 steps 2, 3; Eq. (2))
//  k_lam   wave-speed maxima of a given state
//  k_dt    global maximum and dt = C h / (d (2N+1) lambda)   (Sec. 3 "Time stepping")
//
// k_pred mapping.  One workgroup holds CPB cells, one thread per spatial node
// ("node role").  The node thread keeps the time column of its node q[t][v]
// and the Picard accumulator in registers.  Spatial contractions need a whole
// pencil along axis i: per batch of S time slices the node threads publish
// q into LDS, then every thread takes "pencil tasks" (one time slice, one
// pencil along axis i): it evaluates F_i at the n pencil nodes and contracts
// with D (n^2 m FMAs from n m LDS reads), summing into an LDS slice buffer.
// The node thread then applies the time operator P from registers.  The
// space-time tensor never reaches HBM (Theorem 1): only the 2d face traces
// (time-integrated) and Q~ = Q + dt V are written.
#pragma once

#include "common.hpp"

namespace adg {

// ST_: the hull keeps the traces at every time node (Table 1's extrapolate
// cardinality) and the Riemann problems are solved per time node; otherwise
// the traces are time-integrated (one time value per face node).
// MX_: the bfloat16 predictor (float arithmetic, the Picard contractions on
// the matrix cores with bfloat16 inputs; Real_ must be float).
template <int D_, int N_, template <int> class PDET, class Real_, bool ST_ = false,
          bool MX_ = false>
struct Fwd {
  static constexpr int D = D_, N = N_, n = N_ + 1;
  static constexpr bool ST = ST_;
  static constexpr bool MX = MX_;
  static constexpr int NT = ST_ ? N_ + 1 : 1;         // time values per trace
  using PDE = PDET<D_>;
  using Real = Real_;
  static constexpr int M = PDE::M, NPAR = PDE::NPAR;
  static constexpr int NS = ipow(n, D), NF = ipow(n, D - 1);
  static constexpr int NQ = PDE::LINEAR ? 1 : 2;
  // predictor block
  static constexpr int CPB = (NS >= 128) ? 1 : 128 / NS;
  static constexpr int NODE_THREADS = CPB * NS;      // one thread per spatial node
  // Threads per cell: one per node; the matrix-core contraction takes every
  // lane of a wave, so a cell gets whole waves (the threads past the nodes
  // only take pencil tasks).
  static constexpr int TPC = (MX_ && CPB == 1) ? (NS + 63) / 64 * 64 : NS;
  static constexpr int THREADS = CPB * TPC;
  static_assert(!MX_ || (THREADS % 64 == 0 && std::is_same<Real_, float>::value && !ST_),
                "the matrix-core predictor needs whole waves and float arithmetic");
  // LDS slice layout, as planes indexed by the slot e = tt * NSP + node of a
  // buffer of NSL time slices.  Packed: the variables in groups of VEC
  // (2 float64, 4 float) in 16-byte planes [group][slice][node] and the
  // remaining ones in planes of one variable [var][slice][node], so a node's
  // values move as 16-byte words.  Otherwise one plane per variable.
  // float64 is always packed; float is packed for the linear PDEs (measured
  // faster there, slower for Euler, whose float kernel pairs its 4-byte
  // accesses as it is).  Slices are not padded: a slice stride that is a
  // multiple of 64 words (the float C2 stride padded by 3 was 128) puts the
  // two time slices of a paired access on one bank.  The pencil tasks are
  // dealt to the lanes in the order of TaskOrder below, which keeps every
  // pencil access free of bank conflicts.
  static constexpr bool DBL = std::is_same<Real, double>::value;
  static constexpr int VEC = DBL ? 2 : 4;               // values per 16-byte word
  static constexpr int NV = M / VEC;                    // 16-byte words per node
  static constexpr bool PACKED = DBL || (NV > 0 && PDE::LINEAR);
  // Slots of a slice: node (x, rest) sits at slot x + XP * rest.  When n is a
  // multiple of 4 every x-row is padded to n + 1 slots: the pencils along x
  // then start n + 1 slots apart, an odd stride, where n apart would put
  // gcd(n, 16) lanes of a 16-lane access on one bank (4-way at n = 4, 8-way
  // at n = 8; the 2-way case n = 6 is cheaper than the padding).
  static constexpr int XP = (n % 4 == 0) ? n + 1 : n;
  // Long float64 time columns (n >= 7, nonlinear flux): each Picard
  // iteration gathers sum_i D_i F_i slice by slice at the node threads
  // instead of the pencil tasks (see pred_cell).
  static constexpr bool GATHER = !(PDE::LINEAR && !ST_ && !MX_) && !MX_ && DBL && n >= 7;
  static constexpr int NSLOT = XP * NF;
  __host__ __device__ static constexpr int slot(int node) { return (node % n) + XP * (node / n); }
  __host__ __device__ static constexpr int sstride(int I) { return I == 0 ? 1 : XP * ipow(n, I - 1); }
  static constexpr int NSP = NSLOT;
  static constexpr int MP = M;
  template <int NSL>
  __device__ static __forceinline__ int lidx_e(int e, int v) {
    if constexpr (PACKED) {
      if (v < NV * VEC) return ((v / VEC) * NSL * NSP + e) * VEC + (v % VEC);
      return (NV * VEC + (v - NV * VEC)) * NSL * NSP + e;
    } else {
      return v * NSL * NSP + e;
    }
  }
  __device__ static __forceinline__ int lidx(int tt, int v, int pos);
  // Lanes the LDS serves per pass for this layout's accesses (64 banks of
  // 4 B; measured): reads take 256 bytes per pass (16-byte words 16 lanes,
  // 8-byte words 32, 4-byte words 64), writes 128 bytes (8, 16 and 32
  // lanes).  A group of G lanes is conflict-free when its words are distinct
  // modulo G.
  // Axis sums of a pencil (n m values): all reads before the writes, except
  // for large float pencils, where the extra live values cost more waves
  // than the serialised node-by-node read-modify-write.
  static constexpr bool READ_FIRST = DBL || n * M <= 32;
  static constexpr int NGROUP = PACKED ? 3 : 2;
  static constexpr int group(int c) {
    return PACKED ? (c == 0 ? 8 : (c == 1 ? 16 : (DBL ? 32 : 64))) : (c == 0 ? 32 : 64);
  }
  static constexpr int FIN_BYTES = (D + 2) * NS * M * 8;                 // Fbar_i, qbar, V
                                                                          // (or q, F_i at one time node)
  // Picard slices: up to 80 KiB, or as much as the finalisation needs anyway.
  static constexpr int LDS_BUDGET = FIN_BYTES > 80 * 1024 ? FIN_BYTES : 80 * 1024;
  static constexpr int SLICE_BYTES = 2 * NSP * MP * (int)sizeof(Real);
  static constexpr int pick_S() {
    for (int s = n; s > 1; --s)
      if (CPB * s * SLICE_BYTES <= LDS_BUDGET) return s;
    return 1;
  }
  // ALIAS: one LDS buffer holds all n slices; every thread first contracts
  // its pencils of all d axes into registers, then the axis sums overwrite
  // the buffer in place (half the LDS of a separate rhs buffer).
  static constexpr int FULL_BYTES = CPB * n * NSP * MP * (int)sizeof(Real);
  static constexpr bool ALIAS = 2 * FULL_BYTES > 32 * 1024 && FULL_BYTES <= 48 * 1024;
  static constexpr int S = ALIAS ? n : pick_S();
  static constexpr int NB = (n + S - 1) / S;                 // batches per iteration
  static constexpr int PIC_BYTES = (ALIAS ? 1 : 2) * S * NSP * MP * (int)sizeof(Real);
  static constexpr int FIRST_BYTES = D * NSP * MP * (int)sizeof(Real);   // d flux planes of u
  static constexpr int max3(int x, int y, int z) { return x > y ? (x > z ? x : z) : (y > z ? y : z); }
  // Linear flux: the predictor as powers of the spatial operator (no time
  // slices in LDS; see pred_cell).  Not for the matrix-core form, whose
  // rounding of the Picard contractions' inputs is part of its definition.
  static constexpr bool CK = PDE::LINEAR && !ST_ && !MX_;
  static_assert(!(GATHER && (ALIAS || CK)), "the gather form replaces the batched pencils only");
  // gather form: flux planes of two slices, used in turn
  // linear flux: the finalisation takes Fbar_i = F_i(qbar) one axis at a
  // time (qbar, V and one flux plane)
  static constexpr int FIN_CK_BYTES = 3 * NS * M * 8;
  static constexpr int MAIN_BYTES =
      GATHER ? (2 * FIRST_BYTES > FIN_BYTES ? 2 * FIRST_BYTES : FIN_BYTES)
      : CK ? (FIRST_BYTES > FIN_CK_BYTES ? FIRST_BYTES : FIN_CK_BYTES) : max3(PIC_BYTES, FIRST_BYTES, FIN_BYTES);
  // n >= 7: the gathers read D from LDS.  Indexing the kernel argument's
  // table by a lane-dependent row makes the compiler copy the whole
  // argument block to scratch memory at that size, and every table read
  // (also the uniform ones) then goes through scratch.
  static constexpr bool DLDS = n >= 7;
  static constexpr int DTAB_OFF = (MAIN_BYTES + 15) / 16 * 16;
  static constexpr int DROW = n + 1;                 // D rows padded: 8 rows n apart share banks
  // linear flux: the power-form coefficients (KTab::beta) in LDS
  static constexpr int BTAB_OFF = DTAB_OFF + (DLDS ? n * DROW * 8 : 0);
  static constexpr int CELL_BYTES = (BTAB_OFF + (CK ? KTab<n, Real>::BK * 8 : 0) + 15) / 16 * 16;
  static constexpr int LDS_BYTES = CPB * CELL_BYTES;
  static_assert(LDS_BYTES <= 160 * 1024, "predictor LDS exceeds the CU's 160 KiB");
  // per cell; layout [face][time][qty][var][face node] (face nodes fastest:
  // a wave writes and reads consecutive face nodes of one variable)
  static constexpr int64_t TRACE_ELEMS = 2LL * D * NT * NQ * NF * M;
  static constexpr int64_t TFACE = (int64_t)NT * NQ * NF * M;   // one face
  // corrector block: one thread per face task and per node
  static constexpr int FT = 2 * D * NF;
  static constexpr int CT = NS > FT ? NS : FT;
  static constexpr int CCPB = (CT >= 128) ? 1 : 128 / CT;
  static constexpr int CTHREADS = CCPB * CT;
  static constexpr int CORR_CELL_BYTES = (2 * D * NF * (M + NT) + 2 * D * NT + (n >= 7 ? 2 * n : 0)) * 8;
};

template <int D_, int N_, template <int> class PDET, class Real_, bool ST_, bool MX_>
__device__ __forceinline__ int Fwd<D_, N_, PDET, Real_, ST_, MX_>::lidx(int tt, int v, int pos) {
  return lidx_e<S>(tt * NSP + slot(pos), v);
}

// Lane order of the pencil tasks of one axis for a batch of ns time slices.
// Task (tt, b) is the pencil along axis I through face node b at slice tt; a
// lane reads and writes the slots e0 + j n^I, j = 0..n-1, with e0 its first
// node.  Greedy order: each lane takes the first unused task whose e0 is
// distinct, modulo G, from the e0 of the lanes before it in its aligned
// group of G lanes, for every G the layout's reads and writes are served in
// (the last constraints dropped first when none fits).  The offsets j n^I are the same on every
// lane, so one order serves the whole pencil.
template <int T>
struct TaskOrder {
  unsigned short e0[T];
};

template <class K, int ns, int I>
constexpr TaskOrder<ns * K::NF> make_task_order() {
  constexpr int n = K::n, NF = K::NF, T = ns * NF, s = ipow(n, I);
  TaskOrder<T> r{};
  int off[T] = {};
  bool used[T] = {};
  for (int task = 0; task < T; ++task) {
    const int tt = task / NF, b = task % NF;
    off[task] = tt * K::NSP + K::slot((b % s) + s * n * (b / s));
  }
  unsigned long long mask[3] = {0ull, 0ull, 0ull};
  for (int lane = 0; lane < T; ++lane) {
    for (int c = 0; c < K::NGROUP; ++c)
      if (lane % K::group(c) == 0) mask[c] = 0ull;
    int pick = -1;
    for (int keep = K::NGROUP; keep >= 0 && pick < 0; --keep) {
      for (int k = 0; k < T && pick < 0; ++k) {
        if (used[k]) continue;
        bool ok = true;
        for (int c = 0; c < keep; ++c)
          if ((mask[c] >> (off[k] % K::group(c))) & 1ull) ok = false;
        if (ok) pick = k;
      }
    }
    used[pick] = true;
    for (int c = 0; c < K::NGROUP; ++c) mask[c] |= 1ull << (off[pick] % K::group(c));
    r.e0[lane] = (unsigned short)off[pick];
  }
  return r;
}

template <class K, int ns, int I>
__constant__ TaskOrder<ns * K::NF> task_order = make_task_order<K, ns, I>();

// First slot of this lane's pencil task (0 for lanes without a task).
template <class K, int ns, int I>
__device__ __forceinline__ int task_e0(int a) {
  return a < ns * K::NF ? (int)task_order<K, ns, I>.e0[a] : 0;
}

template <class K>
struct PredP {
  const double* Qin;     // Q (cell, node, var)
  double* Qout;          // Q~ = Q + dt V; may be Qin; null: traces only
  const double* par;
  const double* dt;
  typename K::Real* tr;
  int64_t ncells;
  double inv_h;
  int R;
  Gconst<typename K::Real> g;
  Gconst<double> gd;     // the same constants in float64 (float64 finalisation)
  KTab<K::n, typename K::Real> t;
};

// Predictor of one cell, called by all K::NS node threads of the cell (and
// every thread of the workgroup, for the barriers).  u is this node's state;
// base is the cell's K::CELL_BYTES of LDS.  Writes the cell's face hull and
// Q~ = u + dt V (predict, extrapolate, integrateVolume).
template <class K>
__device__ __forceinline__ void pred_cell(const PredP<K>& p, unsigned char* base, int a,
                                          int64_t cell, bool live, const double (&u)[K::M]) {
  using Real = typename K::Real;
  using PDE = typename K::PDE;
  constexpr int n = K::n, M = K::M, NS = K::NS, NF = K::NF, S = K::S, D = K::D;
  constexpr int NSP = K::NSP;
  const int64_t cs = live ? cell : 0;
  Real* Qs = reinterpret_cast<Real*>(base);      // published slices
  Real* Rs = Qs + S * NSP * K::MP;               // sum_i D_i F_i of the slices

  const double cdt = (*p.dt) * p.inv_h;   // dt / h
  const Real c = (Real)cdt;
  const auto cp = PDE::template cell<Real>(p.par + cs * K::NPAR);

  Real q[n][M];
#pragma unroll
  for (int t = 0; t < n; ++t)
#pragma unroll
    for (int v = 0; v < M; ++v) q[t][v] = (Real)u[v];
  // Node role (publish, time operator, finalisation) on the first NS
  // threads of the cell; threads past them (whole waves for the matrix
  // cores) only take pencil tasks.
  const bool node = (K::TPC == NS) || a < NS;
  const int pa = node ? a : 0;
  // Matrix-core operands of this lane (bfloat16 predictor).
  [[maybe_unused]] MxOps<n> mx;
  if constexpr (K::MX) mx = make_mx_ops<n>(p.t);
  // First slot of this lane's pencil task for each batch size used and axis.
  constexpr int TAIL = n - (K::NB - 1) * S;
  int ordF[D], ordS[D], ordT[D];
  static_for<0, D>([&](auto I_) {
    constexpr int I = decltype(I_)::value;
    ordF[I] = task_e0<K, 1, I>(a);
    ordS[I] = task_e0<K, S, I>(a);
    ordT[I] = (TAIL != S && TAIL != 1) ? task_e0<K, TAIL, I>(a) : 0;
  });
  auto e0_of = [&](auto NS_, auto I_) -> int {
    constexpr int ns = decltype(NS_)::value, I = decltype(I_)::value;
    if constexpr (ns == 1) return ordF[I];
    else if constexpr (ns == S) return ordS[I];
    else return ordT[I];
  };

  // Node role: publish time slices [t0, t0 + ns) of this node's column in
  // the PDE's publish form.
  auto publish = [&](auto T0_, auto NS_) {
    constexpr int t0 = decltype(T0_)::value, ns = decltype(NS_)::value;
    if (!node) return;
#pragma unroll
    for (int tt = 0; tt < ns; ++tt) {
      Real w[M];
      PDE::pub(q[t0 + tt], w, p.g);
#pragma unroll
      for (int v = 0; v < M; ++v) Qs[K::lidx(tt, v, pa)] = w[v];
    }
  };
  // Pencil role: for every published slice and axis I, evaluate F_I along a
  // pencil and contract with D; the three axis results are summed in Rs.
  auto contract = [&](auto NS_) {
    constexpr int ns = decltype(NS_)::value;
    static_for<0, D>([&](auto I_) {
      constexpr int I = decltype(I_)::value;
      constexpr int sI = K::sstride(I);
      auto pencil = [&](int e0, bool wr) {
        Real out[n][M];
        auto flux_at = [&](int j, Real (&F)[M]) {
          Real qn[M];
#pragma unroll
          for (int v = 0; v < M; ++v) qn[v] = Qs[K::template lidx_e<S>(e0 + j * sI, v)];
          PDE::template flux_pub<I>(qn, F, p.g, cp);
        };
        if constexpr (K::MX) pencil_dF_mx<n, M>(mx, flux_at, out);
        else pencil_dF<n, M, Real>(p.t, flux_at, out);
        if (!wr) return;
        // axis sums: for small pencils every read before any write, so the
        // reads are not serialised behind possibly aliasing stores; large
        // ones node by node (fewer live registers)
        if constexpr (I > 0 && K::READ_FIRST) {
#pragma unroll
          for (int k = 0; k < n; ++k)
#pragma unroll
            for (int v = 0; v < M; ++v) out[k][v] += Rs[K::template lidx_e<S>(e0 + k * sI, v)];
        }
#pragma unroll
        for (int k = 0; k < n; ++k)
#pragma unroll
          for (int v = 0; v < M; ++v) {
            if constexpr (I > 0 && !K::READ_FIRST) out[k][v] += Rs[K::template lidx_e<S>(e0 + k * sI, v)];
            Rs[K::template lidx_e<S>(e0 + k * sI, v)] = out[k][v];
          }
      };
      if constexpr (K::MX) {
        // every lane takes part in the matrix-core contraction; lanes
        // without a task contract a valid pencil and discard it
        pencil(e0_of(NS_, I_), a < ns * NF);
      } else if (ns * NF == NS || a < ns * NF) {
        pencil(e0_of(NS_, I_), true);             // at most one task per thread
      }
      __syncthreads();
    });
  };

  // First iteration: q = u on every time node, so sum_i D_i F_i(q) is the
  // same on every slice and P reduces to its row sums.  Every node thread
  // evaluates its d fluxes of u, then gathers sum_i D_i F_i at its own node
  // from the d pencils through it (all lanes busy, one barrier).  In float
  // the gather subtracts the node's own flux first (zero row sums of D), so
  // that a constant state has exactly zero derivative.
  // rv = sum_i D_i F_i(x) at this node for a field x given per node (every
  // node thread its own value): the node threads write their d fluxes of x,
  // then gather from the d pencils through their node (one barrier before,
  // one after, which frees Fs).
  if constexpr (K::CK) {
    if (a == 0) {
      double* sB = reinterpret_cast<double*>(base + K::BTAB_OFF);
#pragma unroll
      for (int k = 0; k < KTab<n, Real>::BK; ++k) sB[k] = p.t.beta[k];
    }
  }
  // D (the matrix-core form: Dx) in LDS for the gathers (n >= 7)
  [[maybe_unused]] double* sDg = reinterpret_cast<double*>(base + K::DTAB_OFF);
  if constexpr (K::DLDS) {
    // static indices only: a dynamic index into the kernel argument would
    // make the compiler copy the whole argument block to scratch memory
    if (a == 0) {
#pragma unroll
      for (int i = 0; i < n * n; ++i)
        sDg[(i / n) * K::DROW + i % n] = K::MX ? (double)p.t.Dx[i / n][i % n] : (double)p.t.D[i / n][i % n];
    }
  }
  auto gather_L = [&](const Real (&x)[M], Real (&rv)[M]) {
    Real* Fs = reinterpret_cast<Real*>(base);      // [axis][var][node] planes
    constexpr bool REF = !std::is_same<Real, double>::value;
    Real Fo[REF ? D : 1][M];
    if (node) {
      Real w[M];
      PDE::pub(x, w, p.g);
      static_for<0, D>([&](auto I_) {
        constexpr int I = decltype(I_)::value;
        Real F[M];
        PDE::template flux_pub<I>(w, F, p.g, cp);
#pragma unroll
        for (int v = 0; v < M; ++v) {
          Fs[K::template lidx_e<D>(I * NSP + K::slot(pa), v)] = F[v];
          if constexpr (REF) Fo[I][v] = F[v];
        }
      });
    }
    __syncthreads();
#pragma unroll
    for (int v = 0; v < M; ++v) rv[v] = Real(0);
    if (node) static_for<0, D>([&](auto I_) {
      constexpr int I = decltype(I_)::value;
      constexpr int sI = K::sstride(I);
      const int ai = coord<n, I>(pa);
      const int e0 = I * NSP + K::slot(pa) - ai * sI;
      if constexpr (K::MX) {
        // as the matrix-core pencils: x_j = bf16(F_j - F_ref) with the
        // pencil's reference flux, contracted with Dh + Dl (exact in float)
        float F[n][M];
#pragma unroll
        for (int j = 0; j < n; ++j)
#pragma unroll
          for (int v = 0; v < M; ++v) F[j][v] = Fs[K::template lidx_e<D>(e0 + j * sI, v)];
#pragma unroll
        for (int v = 0; v < M; ++v) {
          const float Fr = pencil_ref<n, M>(F, v);
#pragma unroll
          for (int j = 0; j < n; ++j) {
            const float x = (float)(__bf16)(F[j][v] - Fr);
            rv[v] = fma(K::DLDS ? (float)sDg[ai * K::DROW + j] : p.t.Dx[ai][j], x, rv[v]);
          }
        }
      } else {
#pragma unroll
        for (int j = 0; j < n; ++j) {
          const Real dj = K::DLDS ? (Real)sDg[ai * K::DROW + j] : p.t.D[ai][j];
#pragma unroll
          for (int v = 0; v < M; ++v) {
            const Real F = Fs[K::template lidx_e<D>(e0 + j * sI, v)];
            if constexpr (REF)
              rv[v] = fma(dj, F - Fo[I][v], rv[v]);
            else
              rv[v] = fma(dj, F, rv[v]);
          }
        }
      }
    });
    __syncthreads();                                // Fs is reused after
  };
  // Linear flux: F_i(q) = A_i q with the cell's constant material, so
  // sum_i D_i F_i(x) = sum_i A_i (D_i x): one plane of x in LDS, gathered
  // along the d pencils through the node, then the flux of each axis applied
  // to its gathered derivative at the node (a third of the LDS writes of
  // gather_L).  float: the derivative of x - x_node (D's rows sum to zero),
  // so a constant field has exactly zero derivative.
  [[maybe_unused]] auto gather_Lx = [&](const Real (&x)[M], Real (&rv)[M]) {
    Real* Xs = reinterpret_cast<Real*>(base);      // [var][node] plane
    constexpr bool REF = !std::is_same<Real, double>::value;
    if (node) {
#pragma unroll
      for (int v = 0; v < M; ++v) Xs[K::template lidx_e<1>(K::slot(pa), v)] = x[v];
    }
    __syncthreads();
#pragma unroll
    for (int v = 0; v < M; ++v) rv[v] = Real(0);
    if (node) static_for<0, D>([&](auto I_) {
      constexpr int I = decltype(I_)::value;
      constexpr int sI = K::sstride(I);
      const int ai = coord<n, I>(pa);
      const int e0 = K::slot(pa) - ai * sI;
      Real g[M];
#pragma unroll
      for (int v = 0; v < M; ++v) g[v] = Real(0);
      // variable by variable: the pencil's n m loads are not all in flight
      // (and live) at once
      Real dr[n];
#pragma unroll
      for (int j = 0; j < n; ++j) dr[j] = K::DLDS ? (Real)sDg[ai * K::DROW + j] : p.t.D[ai][j];
#pragma unroll
      for (int v = 0; v < M; ++v) {
#pragma unroll
        for (int j = 0; j < n; ++j) {
          const Real xv = Xs[K::template lidx_e<1>(e0 + j * sI, v)];
          g[v] = fma(dr[j], REF ? xv - x[v] : xv, g[v]);
        }
      }
      Real F[M];
      PDE::template flux<I>(g, F, p.g, cp);
#pragma unroll
      for (int v = 0; v < M; ++v) rv[v] += F[v];
    });
    __syncthreads();                                // Xs is reused after
  };
  auto first_iteration = [&]() {
    Real uu[M], rv[M];
#pragma unroll
    for (int v = 0; v < M; ++v) uu[v] = (Real)u[v];
    gather_L(uu, rv);
#pragma unroll
    for (int v = 0; v < M; ++v)
#pragma unroll
      for (int t = 0; t < n; ++t) q[t][v] = (Real)u[v] - c * (p.t.Ps[t] * rv[v]);
  };

  // ---- predict: Picard iteration q <- u - (dt/h) P sum_i D_i F_i(q) ----
  [[maybe_unused]] double qbar_ck[M];
  if constexpr (K::CK) {
    // Linear flux: rhs(q) = L q slice by slice, L = sum_i D_i F_i, so from
    // q^0 = 1 (x) u the iterates are q^r = sum_{k<=r} (-c)^k T_k (x) L^k u
    // with T_0 = 1, T_k = P^{k-1} Ps (the time operator commutes with L),
    // exactly, R applications of L to one spatial field instead of R sweeps
    // over the n time slices.  The finalisation needs only the time average
    // qbar = sum_k (-c)^k (w . T_k) L^k u (linear fluxes: Fbar = F(qbar)).
    Real vk[M];
    const double* sB = reinterpret_cast<const double*>(base + K::BTAB_OFF);
#pragma unroll
    for (int v = 0; v < M; ++v) {
      vk[v] = (Real)u[v];
      qbar_ck[v] = u[v];
    }
    double ck = 1.0;
    // L^k u vanishes for k > d N in exact arithmetic (BK covers that), so
    // iterations past BK would add only products of two rounding residues
    const int RK = p.R < KTab<n, Real>::BK ? p.R : KTab<n, Real>::BK;
    for (int k = 1; k <= RK; ++k) {
      Real rv[M];
      gather_Lx(vk, rv);
      ck *= -cdt;
      const double beta = sB[k - 1];   // w . T_k (written before gather_Lx's barriers)
#pragma unroll
      for (int v = 0; v < M; ++v) {
        vk[v] = rv[v];
        qbar_ck[v] = fma(ck * beta, (double)rv[v], qbar_ck[v]);
      }
    }
  } else if constexpr (K::GATHER) {
    // Every node thread evaluates the d fluxes of its node at one slice and
    // gathers sum_i D_i F_i at that node from the d pencils through it
    // (gather_L, D from LDS); P is applied from registers as the slices
    // arrive.  The pencil form at this size keeps a pencil's n m inputs and
    // outputs live beside the 2 n m values of the time column and its
    // accumulator, which overflows the register file, and runs one axis at
    // a time on n^(d-1) of the n^d threads; the gather uses every node
    // thread and holds m values per slice, at twice the multiply-adds of the
    // even/odd pencils.
    // Two flux-plane buffers used in turn: a thread writes buffer g % 2 for
    // the g-th gather only after the barrier of gather g - 1, which every
    // reader of gather g - 2 (the same buffer) has passed, so one barrier
    // per slice suffices.
    Real* Fb2 = reinterpret_cast<Real*>(base);
    int g = 0;
    auto gather_db = [&](const Real (&x)[M], Real (&rv)[M]) {
      Real* Fs = Fb2 + (g & 1) * (D * NSP * K::MP);
      ++g;
      if (node) {
        Real w[M];
        PDE::pub(x, w, p.g);
        static_for<0, D>([&](auto I_) {
          constexpr int I = decltype(I_)::value;
          Real F[M];
          PDE::template flux_pub<I>(w, F, p.g, cp);
#pragma unroll
          for (int v = 0; v < M; ++v) Fs[K::template lidx_e<D>(I * NSP + K::slot(pa), v)] = F[v];
        });
      }
      __syncthreads();
#pragma unroll
      for (int v = 0; v < M; ++v) rv[v] = Real(0);
      if (node) static_for<0, D>([&](auto I_) {
        constexpr int I = decltype(I_)::value;
        constexpr int sI = K::sstride(I);
        const int ai = coord<n, I>(pa);
        const int e0 = I * NSP + K::slot(pa) - ai * sI;
#pragma unroll
        for (int j = 0; j < n; ++j) {
          const Real dj = (Real)sDg[ai * K::DROW + j];
#pragma unroll
          for (int v = 0; v < M; ++v) rv[v] = fma(dj, Fs[K::template lidx_e<D>(e0 + j * sI, v)], rv[v]);
        }
      });
    };
    first_iteration();
    for (int r = 1; r < p.R; ++r) {
      Real acc[n][M];
#pragma unroll
      for (int t = 0; t < n; ++t)
#pragma unroll
        for (int v = 0; v < M; ++v) acc[t][v] = Real(0);
      static_for<0, n>([&](auto T_) {
        constexpr int tt = decltype(T_)::value;
        Real rv[M];
        gather_db(q[tt], rv);
#pragma unroll
        for (int t = 0; t < n; ++t)
#pragma unroll
          for (int v = 0; v < M; ++v) acc[t][v] = fma(p.t.P[t][tt], rv[v], acc[t][v]);
      });
#pragma unroll
      for (int t = 0; t < n; ++t)
#pragma unroll
        for (int v = 0; v < M; ++v) q[t][v] = (Real)u[v] - c * acc[t][v];
    }
  } else if constexpr (K::ALIAS) {
    // One pencil per axis per thread and slice: evaluate F_I along the
    // pencil, contract with D, keep the result in registers.
    auto pencils = [&](auto NS_, auto& out) {
      constexpr int ns = decltype(NS_)::value;
      const bool act = (ns * NF == NS && K::TPC == NS) || a < ns * NF;
      static_for<0, D>([&](auto I_) {
        constexpr int I = decltype(I_)::value;
        constexpr int sI = K::sstride(I);
        const int e0 = e0_of(NS_, I_);
        auto flux_at = [&](int j, Real (&F)[M]) {
          Real qn[M];
#pragma unroll
          for (int v = 0; v < M; ++v) qn[v] = Qs[K::template lidx_e<S>(e0 + j * sI, v)];
          PDE::template flux_pub<I>(qn, F, p.g, cp);
        };
        // matrix cores: every lane takes part (lanes without a task
        // contract a valid pencil and write nothing)
        if constexpr (K::MX) pencil_dF_mx<n, M>(mx, flux_at, out[I]);
        else if (act) pencil_dF<n, M, Real>(p.t, flux_at, out[I]);
      });
      __syncthreads();                              // all pencils read: reuse Qs as rhs
      static_for<0, D>([&](auto I_) {
        constexpr int I = decltype(I_)::value;
        if (act) {
          constexpr int sI = K::sstride(I);
          const int e0 = e0_of(NS_, I_);
          // small pencils: every read before any write (see contract)
          if constexpr (I > 0 && K::READ_FIRST) {
#pragma unroll
            for (int k = 0; k < n; ++k)
#pragma unroll
              for (int v = 0; v < M; ++v) out[I][k][v] += Qs[K::template lidx_e<S>(e0 + k * sI, v)];
          }
#pragma unroll
          for (int k = 0; k < n; ++k)
#pragma unroll
            for (int v = 0; v < M; ++v) {
              if constexpr (I > 0 && !K::READ_FIRST) out[I][k][v] += Qs[K::template lidx_e<S>(e0 + k * sI, v)];
              Qs[K::template lidx_e<S>(e0 + k * sI, v)] = out[I][k][v];
            }
        }
        __syncthreads();
      });
    };
    Real out[D][n][M];
    first_iteration();
    for (int r = 1; r < p.R; ++r) {
      // no barrier before the publish: a node thread reads its own slots'
      // rhs below and overwrites only those same slots here
      publish(std::integral_constant<int, 0>{}, std::integral_constant<int, n>{});
      __syncthreads();
      pencils(std::integral_constant<int, n>{}, out);
#pragma unroll
      for (int v = 0; v < M; ++v) {
        Real rv[n];
#pragma unroll
        for (int tt = 0; tt < n; ++tt) rv[tt] = node ? Qs[K::lidx(tt, v, pa)] : Real(0);
#pragma unroll
        for (int t = 0; t < n; ++t) {
          Real acc = Real(0);
#pragma unroll
          for (int tt = 0; tt < n; ++tt) acc = fma(p.t.P[t][tt], rv[tt], acc);
          q[t][v] = (Real)u[v] - c * acc;
        }
      }
    }
  } else {
  first_iteration();
  for (int r = 1; r < p.R; ++r) {
    Real acc[n][M];
#pragma unroll
    for (int t = 0; t < n; ++t)
#pragma unroll
      for (int v = 0; v < M; ++v) acc[t][v] = Real(0);

    static_for<0, K::NB>([&](auto B_) {
      constexpr int t0 = decltype(B_)::value * S;
      constexpr int ns = (n - t0) < S ? (n - t0) : S;
      if constexpr (K::NB > 1) __syncthreads();   // Qs/Rs reuse across batches
      publish(std::integral_constant<int, t0>{}, std::integral_constant<int, ns>{});
      __syncthreads();
      contract(std::integral_constant<int, ns>{});
#pragma unroll
      for (int tt = 0; tt < ns; ++tt)
#pragma unroll
        for (int v = 0; v < M; ++v) {
          const Real rv = Rs[K::lidx(tt, v, pa)];
#pragma unroll
          for (int t = 0; t < n; ++t) acc[t][v] = fma(p.t.P[t][t0 + tt], rv, acc[t][v]);
        }
    });

#pragma unroll
    for (int t = 0; t < n; ++t)
#pragma unroll
      for (int v = 0; v < M; ++v) q[t][v] = (Real)u[v] - c * acc[t][v];
  }
  }
  __syncthreads();   // LDS is reused below

  // ---- extrapolate + integrateVolume on time averages (float64) ----
  // [axis][var][node]: time-averaged F_i (linear flux: one axis at a time)
  double* Fb = reinterpret_cast<double*>(base);
  double* Qb = Fb + (K::CK ? 1 : D) * NS * M;     // [var][node]: time-averaged q
  double* Vs = Qb + NS * M;                       // [var][node]: volume term
  [[maybe_unused]] const auto cpd = PDE::template cell<double>(p.par + cs * K::NPAR);
  if (node && K::CK) {
    if constexpr (K::CK) {
#pragma unroll
      for (int v = 0; v < M; ++v) Qb[v * NS + a] = qbar_ck[v];
      double F[M];
      PDE::template flux<0>(qbar_ck, F, p.gd, cpd);
#pragma unroll
      for (int v = 0; v < M; ++v) Fb[v * NS + a] = F[v];
    }
  } else if (node) {
    double fb[D][M];
#pragma unroll
    for (int I = 0; I < D; ++I)
#pragma unroll
      for (int v = 0; v < M; ++v) fb[I][v] = 0.0;
#pragma unroll
    for (int v = 0; v < M; ++v) {
      double s = 0.0;
#pragma unroll
      for (int t = 0; t < n; ++t) s += p.t.w[t] * (double)q[t][v];
      Qb[v * NS + a] = s;
    }
#pragma unroll
    for (int t = 0; t < n; ++t) {
      Real w[M];
      PDE::pub(q[t], w, p.g);
      static_for<0, D>([&](auto I_) {
        constexpr int I = decltype(I_)::value;
        Real F[M];
        PDE::template flux_pub<I>(w, F, p.g, cp);
#pragma unroll
        for (int v = 0; v < M; ++v) fb[I][v] += p.t.w[t] * (double)F[v];
      });
    }
#pragma unroll
    for (int I = 0; I < D; ++I)
#pragma unroll
      for (int v = 0; v < M; ++v) Fb[(I * M + v) * NS + a] = fb[I][v];
  }
  __syncthreads();
  static_for<0, D>([&](auto I_) {
    constexpr int I = decltype(I_)::value;
    if constexpr (K::CK && I > 0) {
      // F_I(qbar) into the one flux plane (the previous axis' readers are
      // done: barrier at the end of its tasks)
      if (node) {
        double F[M];
        PDE::template flux<I>(qbar_ck, F, p.gd, cpd);
#pragma unroll
        for (int v = 0; v < M; ++v) Fb[v * NS + a] = F[v];
      }
      __syncthreads();
    }
    const double* FbI = Fb + (K::CK ? 0 : I * M * NS);
    // one (variable, face node) pair per task: traces of q and F_I on both
    // faces normal to I, and the Kv contraction of F_I along the pencil
    for (int task = a; task < M * NF; task += K::TPC) {
      const int v = task / NF, b = task - v * NF;
      double fv[n], vol[n], qL = 0.0, qR = 0.0, fL = 0.0, fR = 0.0;
#pragma unroll
      for (int j = 0; j < n; ++j) {
        const int nd = pencil_node<n, I>(b, j);
        fv[j] = FbI[v * NS + nd];
        const double qv = Qb[v * NS + nd];
        qL += p.t.FL[j] * qv;
        qR += p.t.FR[j] * qv;
        fL += p.t.FL[j] * fv[j];
        fR += p.t.FR[j] * fv[j];
      }
#pragma unroll
      for (int k = 0; k < n; ++k) {
        double sacc = 0.0;
#pragma unroll
        for (int j = 0; j < n; ++j) sacc += p.t.Kv[k][j] * fv[j];
        vol[k] = sacc;
      }
      if constexpr (I > 0) {       // every read before any write
#pragma unroll
        for (int k = 0; k < n; ++k) vol[k] += Vs[v * NS + pencil_node<n, I>(b, k)];
      }
#pragma unroll
      for (int k = 0; k < n; ++k) Vs[v * NS + pencil_node<n, I>(b, k)] = vol[k];
      if (!K::ST && live) {
        Real* tr = p.tr + cs * K::TRACE_ELEMS + v * NF + b;
        Real* tL = tr + (int64_t)(2 * I) * K::TFACE;
        Real* tR = tr + (int64_t)(2 * I + 1) * K::TFACE;
        tL[0] = (Real)qL;
        tR[0] = (Real)qR;
        if constexpr (K::NQ == 2) {
          tL[NF * M] = (Real)fL;
          tR[NF * M] = (Real)fR;
        }
      }
    }
    __syncthreads();
  });
  if (live && node && p.Qout) {
#pragma unroll
    for (int v = 0; v < M; ++v) p.Qout[(cell * NS + a) * M + v] = u[v] + cdt * Vs[v * NS + a];
  }
  if constexpr (K::ST) {
    // ---- extrapolate at every time node (Table 1): q(t) and F_i(q(t)) ----
    double* Ts = reinterpret_cast<double*>(base);   // [slot: q, F_0 .. F_{d-1}][var][node]
    static_for<0, n>([&](auto T_) {
      constexpr int t = decltype(T_)::value;
      __syncthreads();                               // Vs / the last slice read
      if (node) {
#pragma unroll
        for (int v = 0; v < M; ++v) Ts[v * NS + a] = (double)q[t][v];
      }
      if (node) static_for<0, D>([&](auto I_) {
        constexpr int I = decltype(I_)::value;
        if constexpr (K::NQ == 2) {
          Real F[M];
          PDE::template flux<I>(q[t], F, p.g, cp);
#pragma unroll
          for (int v = 0; v < M; ++v) Ts[((1 + I) * M + v) * NS + a] = (double)F[v];
        }
      });
      __syncthreads();
      static_for<0, D>([&](auto I_) {
        constexpr int I = decltype(I_)::value;
        for (int task = a; task < M * NF; task += K::TPC) {
          const int v = task / NF, b = task - v * NF;
          double qL = 0.0, qR = 0.0, fL = 0.0, fR = 0.0;
#pragma unroll
          for (int j = 0; j < n; ++j) {
            const int nd = pencil_node<n, I>(b, j);
            const double qv = Ts[v * NS + nd];
            qL += p.t.FL[j] * qv;
            qR += p.t.FR[j] * qv;
            if constexpr (K::NQ == 2) {
              const double fv = Ts[((1 + I) * M + v) * NS + nd];
              fL += p.t.FL[j] * fv;
              fR += p.t.FR[j] * fv;
            }
          }
          if (live) {
            Real* tr = p.tr + cs * K::TRACE_ELEMS + (int64_t)t * K::NQ * NF * M + v * NF + b;
            Real* tL = tr + (int64_t)(2 * I) * K::TFACE;
            Real* tR = tr + (int64_t)(2 * I + 1) * K::TFACE;
            tL[0] = (Real)qL;
            tR[0] = (Real)qR;
            if constexpr (K::NQ == 2) {
              tL[NF * M] = (Real)fL;
              tR[NF * M] = (Real)fR;
            }
          }
        }
      });
    });
  }
}

template <class K>
__global__ void __launch_bounds__(K::THREADS) k_pred(const PredP<K> p) {
  constexpr int M = K::M, NS = K::NS;
  __shared__ __align__(16) unsigned char smem[K::LDS_BYTES];
  const int lc = threadIdx.x / K::TPC;
  const int a = threadIdx.x - lc * K::TPC;
  const int64_t cell = (int64_t)blockIdx.x * K::CPB + lc;
  const bool live = cell < p.ncells;
  const int64_t cs = live ? cell : 0;
  const int an = a < NS ? a : 0;           // threads past the nodes load node 0 (unused)
  double u[M];
#pragma unroll
  for (int v = 0; v < M; ++v) u[v] = p.Qin[(cs * NS + an) * M + v];
  pred_cell<K>(p, smem + lc * K::CELL_BYTES, a, cell, live, u);
}

// ---------------------------------------------------------------------------
// Block-wide maximum of non-negative doubles; result valid in thread 0.
template <int THREADS>
__device__ __forceinline__ double block_max(double x, double* red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x = fmax(x, __shfl_xor(x, o, 64));
  constexpr int NW = (THREADS + 63) / 64;
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) red[w] = x;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NW; ++k) r = fmax(r, red[k]);
  }
  __syncthreads();
  return r;
}

template <class K>
struct CorrP {
  const double* Qin;     // Q~ (cell, node, var)
  double* Qout;          // Q(T + dt); may be Qin
  const double* par;
  const double* dt;
  const typename K::Real* tr;
  double* partial;
  int32_t* flag;
  int64_t ncells;
  int nc[3];
  int brick[3];
  double inv_h;
  Gconst<double> g;
  double LL[K::n], LR[K::n];
  double w[K::n];        // Gauss-Legendre weights (time integral of space-time fluxes)
  double* stf;           // space-time traces, two-pass corrector: time-integrated
                         // F* of every cell's d lower faces [cell][i][var][b]
};

// Cell visited at position g of a brick-major walk of the grid (bricks of
// brick[0] x brick[1] x brick[2] cells, each dividing the grid).
__device__ __forceinline__ int64_t brick_cell(int64_t g, const int* nc, const int* br) {
  const int64_t bs = (int64_t)br[0] * br[1] * br[2];
  const int64_t bi = g / bs, l = g - bi * bs;
  const int64_t nbx = nc[0] / br[0], nby = nc[1] / br[1];
  const int64_t bx = bi % nbx, by = (bi / nbx) % nby, bz = bi / (nbx * nby);
  const int64_t lx = l % br[0], ly = (l / br[0]) % br[1], lz = l / ((int64_t)br[0] * br[1]);
  return (bx * br[0] + lx) + nc[0] * ((by * br[1] + ly) + (int64_t)nc[1] * (bz * br[2] + lz));
}

// One cell group per workgroup.  Workgroup k runs on XCD k mod 8; each XCD
// takes one contiguous eighth of the walk in dispatch order, so the traces
// of recently corrected neighbours are still in its L2.
__device__ __forceinline__ int64_t xcd_group(int64_t groups) {
  const int64_t span = (groups + 7) / 8;
  return (int64_t)(blockIdx.x % 8) * span + blockIdx.x / 8;
}

template <class K>
__device__ __forceinline__ int64_t neighbour(int64_t cell, int i, int dir, const int* nc) {
  int64_t ix = cell % nc[0];
  int64_t rest = cell / nc[0];
  int64_t iy = rest % nc[1];
  int64_t iz = rest / nc[1];
  if (i == 0) ix = (ix + dir + nc[0]) % nc[0];
  else if (i == 1) iy = (iy + dir + nc[1]) % nc[1];
  else iz = (iz + dir + nc[2]) % nc[2];
  return ix + nc[0] * (iy + nc[1] * iz);
}

// Corrector of one cell with NT threads per cell (t = 0..NT-1; all threads
// of the workgroup call it, for the barriers).  solveRiemann on the 2d faces
// (one task per face node), integrateFace + update for node t < NS: the new
// state of node t in Qn, its largest directional speed folded into lmax and
// the admissibility flags into bad (2 also for a face trace whose wave speed
// is not a real number).  lds: the cell's K::CORR_CELL_BYTES.
template <class K, int NTH>
__device__ __forceinline__ void corr_cell(const CorrP<K>& p, double* lds, int t, int64_t cell,
                                          bool live, double (&Qn)[K::M], double& lmax, int& bad) {
  using Real = typename K::Real;
  using PDE = typename K::PDE;
  constexpr int n = K::n, M = K::M, NS = K::NS, NF = K::NF, D = K::D, FT = K::FT;
  constexpr int TPT = (FT + NTH - 1) / NTH;               // face tasks per thread
  constexpr bool EARLY_Q = TPT > 1;                       // see the time-integrated branch
  double* lam = lds;                                     // [2D][NT][NF]
  double* Fs = lam + 2 * D * NF * K::NT;                 // [2D][NF][M]
  double* sm = Fs + 2 * D * NF * M;                      // [2D][NT]
  // n >= 7: LL and LR in LDS (see DLDS), read after the face barriers
  [[maybe_unused]] double* sLf = sm + 2 * D * K::NT;
  if constexpr (K::DLDS) {
    if (t == 0) {
#pragma unroll
      for (int kk = 0; kk < n; ++kk) {
        sLf[kk] = p.LL[kk];
        sLf[n + kk] = p.LR[kk];
      }
    }
  }
  const double cdt = (*p.dt) * p.inv_h;
  if constexpr (K::ST) {
    // Space-time traces: every trace is read once.  The time loop of each
    // face task takes the speeds (for one s per face and time node), the
    // time integral of the mean flux sum_t w_t (fL + fR) / 2 and keeps the
    // jumps qR - qL in registers; once the maxima are known, the dissipation
    // sum_t w_t s_t (qR - qL) / 2 is subtracted: F* integrated in time.
    constexpr int NT = K::NT;
    double acc[TPT][M], dq[TPT][NT][M];
#pragma unroll
    for (int v = 0; v < M; ++v) Qn[v] = 1.0;
#pragma unroll
    for (int r = 0; r < TPT; ++r) {
      const int task = t + r * NTH;
#pragma unroll
      for (int v = 0; v < M; ++v) acc[r][v] = 0.0;
      if (live && task < FT) {
        const int f = task / NF, b = task - f * NF;
        const int i = f >> 1, s = f & 1;
        const int64_t cL = s ? cell : neighbour<K>(cell, i, -1, p.nc);
        const int64_t cR = s ? neighbour<K>(cell, i, +1, p.nc) : cell;
        const auto pL = PDE::template cell<double>(p.par + cL * K::NPAR);
        const auto pR = PDE::template cell<double>(p.par + cR * K::NPAR);
        const Real* trL0 = p.tr + cL * K::TRACE_ELEMS + (int64_t)(2 * i + 1) * K::TFACE + b;
        const Real* trR0 = p.tr + cR * K::TRACE_ELEMS + (int64_t)(2 * i) * K::TFACE + b;
#pragma unroll
        for (int tt = 0; tt < NT; ++tt) {
          const Real* trL = trL0 + (int64_t)tt * K::NQ * NF * M;
          const Real* trR = trR0 + (int64_t)tt * K::NQ * NF * M;
          double qL[M], qR[M], fL[M], fR[M];
#pragma unroll
          for (int v = 0; v < M; ++v) {
            qL[v] = (double)trL[v * NF];
            qR[v] = (double)trR[v * NF];
            if constexpr (K::NQ == 2) {
              fL[v] = (double)trL[NF * M + v * NF];
              fR[v] = (double)trR[NF * M + v * NF];
            }
          }
          double l = 0.0;
          static_for<0, D>([&](auto I_) {
            constexpr int I = decltype(I_)::value;
            if (i == I) {
              if constexpr (K::NQ == 1) {
                PDE::template flux<I>(qL, fL, p.g, pL);
                PDE::template flux<I>(qR, fR, p.g, pR);
              }
              l = fmax(PDE::template speed<I>(qL, p.g, pL), PDE::template speed<I>(qR, p.g, pR));
            }
          });
          if (!(l >= 0.0)) bad |= 2;
          lam[(f * NT + tt) * NF + b] = l;
          const double hw = 0.5 * p.w[tt];
#pragma unroll
          for (int v = 0; v < M; ++v) {
            acc[r][v] += hw * (fL[v] + fR[v]);
            dq[r][tt][v] = qR[v] - qL[v];
            // computed here, not sunk past the barrier below (which would
            // keep every time node's loaded traces live instead)
            asm volatile("" : "+v"(acc[r][v]), "+v"(dq[r][tt][v]));
          }
          // one time node's loads at a time: the kept jumps already hold
          // NT M registers per task
          __builtin_amdgcn_sched_barrier(0);
        }
      }
    }
    __syncthreads();
    for (int ft = t; ft < 2 * D * NT; ft += NTH) {
      if (live) {
        double sv = 0.0;
        for (int b = 0; b < NF; ++b) sv = fmax(sv, lam[ft * NF + b]);
        sm[ft] = sv;
      }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < TPT; ++r) {
      const int task = t + r * NTH;
      if (live && task < FT) {
        const int f = task / NF;
#pragma unroll
        for (int tt = 0; tt < NT; ++tt) {
          const double hs = 0.5 * p.w[tt] * sm[f * NT + tt];
#pragma unroll
          for (int v = 0; v < M; ++v) acc[r][v] -= hs * dq[r][tt][v];
        }
#pragma unroll
        for (int v = 0; v < M; ++v) Fs[task * M + v] = acc[r][v];
      }
    }
    __syncthreads();
    if (live && t < NS) {
      const double* Qp = p.Qin + (cell * NS + t) * M;
#pragma unroll
      for (int v = 0; v < M; ++v) Qn[v] = Qp[v];
    }
  } else {
  // Every load of the cell first (the face traces of all of this thread's
  // tasks and, with several tasks per thread, the node's Q~), so that their
  // latencies overlap.  With one task per thread (NTH >= FT) the Q~ load
  // waits for the update: fewer live registers, more waves for k_corr.
  double qL[TPT][M], qR[TPT][M], fL[TPT][M], fR[TPT][M];
  int64_t cLr[TPT], cRr[TPT];
#pragma unroll
  for (int r = 0; r < TPT; ++r) {
    const int task = t + r * NTH;
    cLr[r] = cRr[r] = 0;
    if (live && task < FT) {
      const int f = task / NF, b = task - f * NF;
      const int i = f >> 1, s = f & 1;
      const int64_t cL = s ? cell : neighbour<K>(cell, i, -1, p.nc);
      const int64_t cR = s ? neighbour<K>(cell, i, +1, p.nc) : cell;
      cLr[r] = cL;
      cRr[r] = cR;
      const Real* trL = p.tr + cL * K::TRACE_ELEMS + (int64_t)(2 * i + 1) * K::NQ * NF * M + b;
      const Real* trR = p.tr + cR * K::TRACE_ELEMS + (int64_t)(2 * i) * K::NQ * NF * M + b;
#pragma unroll
      for (int v = 0; v < M; ++v) {
        qL[r][v] = (double)trL[v * NF];
        qR[r][v] = (double)trR[v * NF];
        if constexpr (K::NQ == 2) {
          fL[r][v] = (double)trL[NF * M + v * NF];
          fR[r][v] = (double)trR[NF * M + v * NF];
        }
      }
    }
  }
#pragma unroll
  for (int v = 0; v < M; ++v) Qn[v] = 1.0;
  if (EARLY_Q && live && t < NS) {
    const double* Qp = p.Qin + (cell * NS + t) * M;
#pragma unroll
    for (int v = 0; v < M; ++v) Qn[v] = Qp[v];
  }
  double fh[TPT][M], dq[TPT][M];
#pragma unroll
  for (int r = 0; r < TPT; ++r) {
    const int task = t + r * NTH;
    if (live && task < FT) {
      const int f = task / NF;
      const int i = f >> 1;
      const auto pL = PDE::template cell<double>(p.par + cLr[r] * K::NPAR);
      const auto pR = PDE::template cell<double>(p.par + cRr[r] * K::NPAR);
      double l = 0.0;
      static_for<0, D>([&](auto I_) {
        constexpr int I = decltype(I_)::value;
        if (i == I) {
          if constexpr (K::NQ == 1) {
            PDE::template flux<I>(qL[r], fL[r], p.g, pL);
            PDE::template flux<I>(qR[r], fR[r], p.g, pR);
          }
          l = fmax(PDE::template speed<I>(qL[r], p.g, pL), PDE::template speed<I>(qR[r], p.g, pR));
        }
      });
#pragma unroll
      for (int v = 0; v < M; ++v) {
        fh[r][v] = 0.5 * (fL[r][v] + fR[r][v]);
        dq[r][v] = qR[r][v] - qL[r][v];
      }
      if (!(l >= 0.0)) bad |= 2;      // a trace without a real wave speed (fmax would skip it)
      lam[task] = l;
    }
  }
  __syncthreads();
  if (live && t < 2 * D) {
    double s = 0.0;
    for (int b = 0; b < NF; ++b) s = fmax(s, lam[t * NF + b]);
    sm[t] = s;
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < TPT; ++r) {
    const int task = t + r * NTH;
    if (live && task < FT) {
      const double hs = 0.5 * sm[task / NF];
#pragma unroll
      for (int v = 0; v < M; ++v) Fs[task * M + v] = fh[r][v] - hs * dq[r][v];
    }
  }
  __syncthreads();
  }
  if (live && t < NS) {
    const int a = t;
    if constexpr (!K::ST && !EARLY_Q) {
      const double* Qp = p.Qin + (cell * NS + a) * M;
#pragma unroll
      for (int v = 0; v < M; ++v) Qn[v] = Qp[v];
    }
    static_for<0, D>([&](auto I_) {
      constexpr int I = decltype(I_)::value;
      const int k = coord<n, I>(a);
      const int b = face_node<n, I>(a);
      const double* Fm = Fs + ((2 * I) * NF + b) * M;
      const double* Fp = Fs + ((2 * I + 1) * NF + b) * M;
      double lr, ll;
      if constexpr (K::DLDS) {
        lr = sLf[n + k];
        ll = sLf[k];
      } else {
        lr = p.LR[k];
        ll = p.LL[k];
      }
#pragma unroll
      for (int v = 0; v < M; ++v) Qn[v] -= cdt * (lr * Fp[v] - ll * Fm[v]);
    });
    const auto pc = PDE::template cell<double>(p.par + cell * K::NPAR);
    static_for<0, D>([&](auto I_) {
      constexpr int I = decltype(I_)::value;
      lmax = fmax(lmax, PDE::template speed<I>(Qn, p.g, pc));
    });
    if (!PDE::admissible(Qn, p.g, pc)) {
      bool fin = true;
#pragma unroll
      for (int v = 0; v < M; ++v) fin = fin && isfinite(Qn[v]);
      bad |= fin ? 2 : 1;
    }
  }
}

template <class K>
__global__ void __launch_bounds__(K::CTHREADS) k_corr(const CorrP<K> p) {
  constexpr int M = K::M, NS = K::NS, CT = K::CT;
  __shared__ double lds[K::CCPB * K::CORR_CELL_BYTES / 8];
  __shared__ double red[(K::CTHREADS + 63) / 64];
  const int lc = threadIdx.x / CT;
  const int t = threadIdx.x - lc * CT;
  const int64_t groups = (p.ncells + K::CCPB - 1) / K::CCPB;
  double lmax = 0.0;
  int bad = 0;
  const int64_t grp = xcd_group(groups);
  if (grp < groups) {                       // uniform over the workgroup
    const int64_t gc = grp * K::CCPB + lc;
    const bool live = gc < p.ncells;
    const int64_t cell = live ? brick_cell(gc, p.nc, p.brick) : 0;
    double Qn[M];
    corr_cell<K, CT>(p, lds + lc * (K::CORR_CELL_BYTES / 8), t, cell, live, Qn, lmax, bad);
    if (live && t < NS) {
      double* Qp = p.Qout + (cell * NS + t) * M;
#pragma unroll
      for (int v = 0; v < M; ++v) Qp[v] = Qn[v];
    }
  }
  const double bm = block_max<K::CTHREADS>(lmax, red);
  if (threadIdx.x == 0) p.partial[blockIdx.x] = bm;
  if (bad && p.flag) atomicOr(p.flag, bad);
}

// Space-time traces, two passes: every face's time-integrated Rusanov flux
// once, then the update.  A single corrector pass reads each hull face twice
// (from both of its cells), and at N+1 time values per face node the hull is
// too large for the second read to find it in L2.
//  k_st_face   a cell takes its d lower faces (its -e_i neighbour's upper
//              face and its own lower face): per face node the time loop
//              of corr_cell's space-time branch (speeds per time node, the
//              time integral of the mean flux, the jumps in registers), the
//              maxima over the face nodes per time node, then
//              F* = sum_t w_t ((fL + fR) / 2 - s_t (qR - qL) / 2), written to
//              stf[cell][i][var][b].  Same operands and order as corr_cell,
//              so the result is the same bit for bit.
//  k_st_update one thread per node: Q~ minus the lifted F* of the node's 2d
//              faces (the lower ones from the cell's own slot, the upper ones
//              from the +e_i neighbours', staged in LDS with coalesced
//              loads), then the speed maxima and flags of the new state as
//              k_corr.
template <class K>
struct StFace {
  static constexpr int FT = K::D * K::NF;
  static constexpr int FCPB = FT >= 256 ? 1 : 256 / FT;
  static constexpr int THREADS = FCPB * FT;
  static constexpr int UCPB = K::NS >= 256 ? 1 : 256 / K::NS;
  static constexpr int UTHREADS = UCPB * K::NS;
};

template <class K>
__global__ void __launch_bounds__(StFace<K>::THREADS) k_st_face(const CorrP<K> p) {
  using PDE = typename K::PDE;
  using Real = typename K::Real;
  constexpr int M = K::M, NF = K::NF, D = K::D, NT = K::NT;
  constexpr int FT = StFace<K>::FT, CC = StFace<K>::FCPB;
  __shared__ double lam[CC][D * NT * NF];
  __shared__ double sm[CC][D * NT];
  const int lc = threadIdx.x / FT;
  const int t = threadIdx.x - lc * FT;
  const int64_t groups = (p.ncells + CC - 1) / CC;
  const int64_t grp = xcd_group(groups);
  if (grp >= groups) return;                    // whole workgroup leaves together
  const int64_t gc = grp * CC + lc;
  const bool live = gc < p.ncells;
  const int64_t cell = live ? brick_cell(gc, p.nc, p.brick) : 0;
  const int i = t / NF, b = t - i * NF;
  int bad = 0;
  double acc[M], dq[NT][M];
#pragma unroll
  for (int v = 0; v < M; ++v) acc[v] = 0.0;
  if (live) {
    const int64_t cL = neighbour<K>(cell, i, -1, p.nc);
    const auto pL = PDE::template cell<double>(p.par + cL * K::NPAR);
    const auto pR = PDE::template cell<double>(p.par + cell * K::NPAR);
    const Real* trL0 = p.tr + cL * K::TRACE_ELEMS + (int64_t)(2 * i + 1) * K::TFACE + b;
    const Real* trR0 = p.tr + cell * K::TRACE_ELEMS + (int64_t)(2 * i) * K::TFACE + b;
#pragma unroll
    for (int tt = 0; tt < NT; ++tt) {
      const Real* trL = trL0 + (int64_t)tt * K::NQ * NF * M;
      const Real* trR = trR0 + (int64_t)tt * K::NQ * NF * M;
      double qL[M], qR[M], fL[M], fR[M];
#pragma unroll
      for (int v = 0; v < M; ++v) {
        qL[v] = (double)trL[v * NF];
        qR[v] = (double)trR[v * NF];
        if constexpr (K::NQ == 2) {
          fL[v] = (double)trL[NF * M + v * NF];
          fR[v] = (double)trR[NF * M + v * NF];
        }
      }
      double l = 0.0;
      static_for<0, D>([&](auto I_) {
        constexpr int I = decltype(I_)::value;
        if (i == I) {
          if constexpr (K::NQ == 1) {
            PDE::template flux<I>(qL, fL, p.g, pL);
            PDE::template flux<I>(qR, fR, p.g, pR);
          }
          l = fmax(PDE::template speed<I>(qL, p.g, pL), PDE::template speed<I>(qR, p.g, pR));
        }
      });
      if (!(l >= 0.0)) bad |= 2;
      lam[lc][(i * NT + tt) * NF + b] = l;
      const double hw = 0.5 * p.w[tt];
#pragma unroll
      for (int v = 0; v < M; ++v) {
        acc[v] += hw * (fL[v] + fR[v]);
        dq[tt][v] = qR[v] - qL[v];
        asm volatile("" : "+v"(acc[v]), "+v"(dq[tt][v]));
      }
      __builtin_amdgcn_sched_barrier(0);       // one time node's loads at a time
    }
  }
  __syncthreads();
  for (int ft = t; ft < D * NT; ft += FT) {
    if (live) {
      double sv = 0.0;
      for (int bb = 0; bb < NF; ++bb) sv = fmax(sv, lam[lc][ft * NF + bb]);
      sm[lc][ft] = sv;
    }
  }
  __syncthreads();
  if (live) {
#pragma unroll
    for (int tt = 0; tt < NT; ++tt) {
      const double hs = 0.5 * p.w[tt] * sm[lc][i * NT + tt];
#pragma unroll
      for (int v = 0; v < M; ++v) acc[v] -= hs * dq[tt][v];
    }
    double* out = p.stf + ((cell * D + i) * M) * NF + b;
#pragma unroll
    for (int v = 0; v < M; ++v) out[v * NF] = acc[v];
  }
  if (bad && p.flag) atomicOr(p.flag, bad);
}

template <class K>
__global__ void __launch_bounds__(StFace<K>::UTHREADS) k_st_update(const CorrP<K> p) {
  using PDE = typename K::PDE;
  constexpr int n = K::n, M = K::M, NS = K::NS, NF = K::NF, D = K::D;
  constexpr int CC = StFace<K>::UCPB, TH = StFace<K>::UTHREADS;
  constexpr int FB = M * NF;                      // one face's F*, contiguous in stf
  // the cell's 2d faces staged with coalesced loads: [lc][2i + s][var][b]
  __shared__ double Fs[CC][2 * D * FB];
  __shared__ int64_t cid[CC];
  __shared__ double red[(TH + 63) / 64];
  const int lc = threadIdx.x / NS;
  const int a = threadIdx.x - lc * NS;
  const int64_t groups = (p.ncells + CC - 1) / CC;
  double lmax = 0.0;
  int bad = 0;
  const int64_t grp = xcd_group(groups);
  if (grp < groups) {                       // uniform over the workgroup
    const int64_t gc = grp * CC + lc;
    const bool live = gc < p.ncells;
    const int64_t cell = live ? brick_cell(gc, p.nc, p.brick) : 0;
    if (a == 0) cid[lc] = live ? cell : -1;
    __syncthreads();
    for (int e = threadIdx.x; e < CC * 2 * D * FB; e += TH) {
      const int c = e / (2 * D * FB), r = e - c * (2 * D * FB);
      const int f = r / FB, k = r - f * FB;
      const int i = f >> 1;
      const int64_t cc = cid[c];
      if (cc >= 0) {
        const int64_t src = (f & 1) ? neighbour<K>(cc, i, +1, p.nc) : cc;
        Fs[c][r] = p.stf[(src * D + i) * FB + k];
      }
    }
    double Qn[M];
    if (live) {
      const double* Qp = p.Qin + (cell * NS + a) * M;
#pragma unroll
      for (int v = 0; v < M; ++v) Qn[v] = Qp[v];
    }
    __syncthreads();
    if (live) {
      const double cdt = (*p.dt) * p.inv_h;
      static_for<0, D>([&](auto I_) {
        constexpr int I = decltype(I_)::value;
        const int k = coord<n, I>(a);
        const int b = face_node<n, I>(a);
        const double* Fm = &Fs[lc][(2 * I) * FB + b];
        const double* Fp = &Fs[lc][(2 * I + 1) * FB + b];
        const double lr = p.LR[k], ll = p.LL[k];
#pragma unroll
        for (int v = 0; v < M; ++v) Qn[v] -= cdt * (lr * Fp[v * NF] - ll * Fm[v * NF]);
      });
      const auto pc = PDE::template cell<double>(p.par + cell * K::NPAR);
      static_for<0, D>([&](auto I_) {
        constexpr int I = decltype(I_)::value;
        lmax = fmax(lmax, PDE::template speed<I>(Qn, p.g, pc));
      });
      if (!PDE::admissible(Qn, p.g, pc)) {
        bool fin = true;
#pragma unroll
        for (int v = 0; v < M; ++v) fin = fin && isfinite(Qn[v]);
        bad |= fin ? 2 : 1;
      }
      double* Qo = p.Qout + (cell * NS + a) * M;
#pragma unroll
      for (int v = 0; v < M; ++v) Qo[v] = Qn[v];
    }
  }
  const double bm = block_max<TH>(lmax, red);
  if (threadIdx.x == 0) p.partial[blockIdx.x] = bm;
  if (bad && p.flag) atomicOr(p.flag, bad);
}

// Shifted and fused step (Sec. 5, Techniques 3 and 4; Alg. 2): per cell the
// corrector of step n (dt of c) and at once the predictor of step n+1 on the
// new state (dt of p), so Q is read and written once per step.  Cells follow
// the corrector's XCD-aware brick walk; K::CPB cells per workgroup with one
// thread per node.  The per-workgroup speed maxima of the new states go to
// c.partial.  run_if (nullable): the rerun of Technique 5, decided on the
// device: the workgroups leave at once unless *run_if != 0, and each takes
// VB cell groups so that a skipped rerun costs few workgroups; a rerun
// leaves the maxima and the flag alone (its corrector repeats the sweep's).
// The sweep itself runs with VB = 1 (no loop, so no registers held across
// cell groups).
template <class K>
struct FusedP {
  CorrP<K> c;
  PredP<K> p;
  const int32_t* run_if;
};

template <class K>
constexpr int fused_cell_bytes() {
  constexpr int cb = (K::CORR_CELL_BYTES + 15) / 16 * 16;
  return K::CELL_BYTES > cb ? K::CELL_BYTES : cb;
}

template <class K, int VB>
__global__ void __launch_bounds__(K::THREADS) k_fused(const FusedP<K> f) {
  constexpr int M = K::M, NS = K::NS, FCB = fused_cell_bytes<K>();
  static_assert(K::CPB * FCB <= 160 * 1024, "fused step LDS exceeds the CU's 160 KiB");
  __shared__ __align__(16) unsigned char smem[K::CPB * FCB];
  __shared__ double red[(K::THREADS + 63) / 64];
  const int lc = threadIdx.x / K::TPC;
  const int a = threadIdx.x - lc * K::TPC;
  const int64_t groups = (f.c.ncells + K::CPB - 1) / K::CPB;
  unsigned char* base = smem + lc * FCB;
  if constexpr (VB == 1) {                  // the sweep: one cell group, maxima and flag
    const int64_t grp = xcd_group(groups);
    const bool act = grp < groups;          // uniform over the workgroup
    const int64_t gc = grp * K::CPB + lc;
    const bool live = act && gc < f.c.ncells;
    const int64_t cell = live ? brick_cell(gc, f.c.nc, f.c.brick) : 0;
    double Qn[M];
    double lmax = 0.0;
    int bad = 0;
    if (act) corr_cell<K, K::TPC>(f.c, reinterpret_cast<double*>(base), a, cell, live, Qn, lmax, bad);
    const double bm = block_max<K::THREADS>(lmax, red);   // ends with a barrier
    if (threadIdx.x == 0) f.c.partial[blockIdx.x] = bm;
    if (bad && f.c.flag) atomicOr(f.c.flag, bad);
    if (act) pred_cell<K>(f.p, base, a, cell, live, Qn);
  } else {                                  // the rerun: VB cell groups, skipped if not due
    if (*f.run_if == 0) return;             // uniform
    const int64_t span = (groups + 7) / 8;  // cell groups per XCD
    for (int vb = 0; vb < VB; ++vb) {
      // virtual workgroup v runs on XCD v mod 8 (gridDim.x is a multiple of 8)
      const int64_t v = blockIdx.x + (int64_t)vb * gridDim.x;
      const int64_t grp = (v % 8) * span + v / 8;             // a bijection of [0, 8 span)
      const bool act = v < 8 * span && grp < groups;          // uniform over the workgroup
      const int64_t gc = grp * K::CPB + lc;
      const bool live = act && gc < f.c.ncells;
      const int64_t cell = live ? brick_cell(gc, f.c.nc, f.c.brick) : 0;
      double Qn[M];
      double lmax = 0.0;
      int bad = 0;
      if (vb > 0) __syncthreads();          // LDS of the previous cell group read
      if (act) corr_cell<K, K::TPC>(f.c, reinterpret_cast<double*>(base), a, cell, live, Qn, lmax, bad);
      __syncthreads();                      // corrector LDS read before reuse
      if (act) pred_cell<K>(f.p, base, a, cell, live, Qn);
    }
  }
}

template <class K>
struct LamP {
  const double* Q;
  const double* par;
  double* partial;
  int64_t ncells;
  Gconst<double> g;
};

template <class K>
__global__ void __launch_bounds__(256) k_lam(const LamP<K> p) {
  using PDE = typename K::PDE;
  constexpr int M = K::M, NS = K::NS, D = K::D;
  __shared__ double red[4];
  const int64_t total = p.ncells * NS;
  double lmax = 0.0;
  for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k < total; k += (int64_t)gridDim.x * 256) {
    const int64_t cell = k / NS;
    double q[M];
#pragma unroll
    for (int v = 0; v < M; ++v) q[v] = p.Q[k * M + v];
    const auto pc = PDE::template cell<double>(p.par + cell * K::NPAR);
    static_for<0, D>([&](auto I_) {
      constexpr int I = decltype(I_)::value;
      lmax = fmax(lmax, PDE::template speed<I>(q, p.g, pc));
    });
  }
  const double bm = block_max<256>(lmax, red);
  if (threadIdx.x == 0) p.partial[blockIdx.x] = bm;
}

// ---------------------------------------------------------------------------
template <class K>
PredP<K> pred_params(const LaunchArgs& a) {
  using Real = typename K::Real;
  PredP<K> p;
  p.Qin = a.qin ? a.qin : a.Q;
  p.Qout = a.traces_only ? nullptr : (a.qout ? a.qout : a.Q);
  p.par = a.params;
  p.dt = a.dt;
  p.tr = reinterpret_cast<Real*>(a.traces);
  p.ncells = a.ncells;
  p.inv_h = a.inv_h;
  p.R = a.R;
  for (int k = 0; k < 4; ++k) {
    p.g.c[k] = (Real)a.gp[k];
    p.gd.c[k] = a.gp[k];
  }
  p.t = make_ktab<K::n, Real>(*a.tab);
  return p;
}

template <class K>
CorrP<K> corr_params(const LaunchArgs& a) {
  CorrP<K> p;
  p.Qin = a.qin ? a.qin : a.Q;
  p.Qout = a.qout ? a.qout : a.Q;
  p.par = a.params;
  p.dt = a.dt;
  p.tr = reinterpret_cast<const typename K::Real*>(a.traces);
  p.partial = a.partial;
  p.flag = a.flag;
  p.ncells = a.ncells;
  for (int k = 0; k < 3; ++k) p.nc[k] = a.nc[k];
  p.inv_h = a.inv_h;
  for (int k = 0; k < 4; ++k) p.g.c[k] = a.gp[k];
  for (int k = 0; k < K::n; ++k) {
    p.LL[k] = a.tab->LL[k];
    p.LR[k] = a.tab->LR[k];
    p.w[k] = a.tab->w[k];
  }
  for (int k = 0; k < 3; ++k) p.brick[k] = a.brick[k];
  p.stf = a.st_face;
  return p;
}

template <class K>
int launch_predict(const LaunchArgs& a) {
  const PredP<K> p = pred_params<K>(a);
  const int64_t blocks = (a.ncells + K::CPB - 1) / K::CPB;
  hipLaunchKernelGGL(k_pred<K>, dim3((unsigned)blocks), dim3(K::THREADS), 0, a.stream, p);
  return (int)hipGetLastError();
}

template <class K>
int64_t reduce_grid(int64_t groups) {
  if (groups < 64) return groups;
  int64_t G = groups < kMaxReduceBlocks ? groups : kMaxReduceBlocks;
  return G - G % 8;
}

template <class K>
int launch_correct(const LaunchArgs& a) {
  const CorrP<K> p = corr_params<K>(a);
  if constexpr (K::ST) {
    if (a.st_face) {
      const int64_t gf = (a.ncells + StFace<K>::FCPB - 1) / StFace<K>::FCPB;
      hipLaunchKernelGGL(k_st_face<K>, dim3((unsigned)(8 * ((gf + 7) / 8))), dim3(StFace<K>::THREADS), 0,
                         a.stream, p);
      hipError_t e = hipGetLastError();
      if (e != hipSuccess) return (int)e;
      const int64_t gu = (a.ncells + StFace<K>::UCPB - 1) / StFace<K>::UCPB;
      const int64_t G = 8 * ((gu + 7) / 8);
      if (G > a.n_partial) return (int)hipErrorInvalidValue;
      *a.n_partial_used = G;
      hipLaunchKernelGGL(k_st_update<K>, dim3((unsigned)G), dim3(StFace<K>::UTHREADS), 0, a.stream, p);
      return (int)hipGetLastError();
    }
  }
  const int64_t groups = (a.ncells + K::CCPB - 1) / K::CCPB;
  const int64_t G = 8 * ((groups + 7) / 8);
  if (G > a.n_partial) return (int)hipErrorInvalidValue;
  *a.n_partial_used = G;
  hipLaunchKernelGGL(k_corr<K>, dim3((unsigned)G), dim3(K::CTHREADS), 0, a.stream, p);
  return (int)hipGetLastError();
}

// Fused step: corrector with a.dt on (qin, traces), predictor with a.dt_pred
// writing (qout, traces_out).
template <class K>
int launch_fused(const LaunchArgs& a) {
  FusedP<K> f;
  f.c = corr_params<K>(a);
  LaunchArgs b = a;
  b.dt = a.dt_pred;
  b.traces = a.traces_out;
  f.p = pred_params<K>(b);
  f.run_if = a.run_if;
  const int64_t groups = (a.ncells + K::CPB - 1) / K::CPB;
  const int64_t G = 8 * ((groups + 7) / 8);             // virtual workgroups
  if (G > a.n_partial) return (int)hipErrorInvalidValue;
  if (a.run_if) {      // a rerun takes 16 cell groups per workgroup
    const int64_t blocks = 8 * ((G / 8 + 15) / 16);
    hipLaunchKernelGGL((k_fused<K, 16>), dim3((unsigned)blocks), dim3(K::THREADS), 0, a.stream, f);
  } else {
    *a.n_partial_used = G;
    hipLaunchKernelGGL((k_fused<K, 1>), dim3((unsigned)G), dim3(K::THREADS), 0, a.stream, f);
  }
  return (int)hipGetLastError();
}

template <class K>
int launch_wave_speed(const LaunchArgs& a) {
  LamP<K> p;
  p.Q = a.Qc;
  p.par = a.params;
  p.partial = a.partial;
  p.ncells = a.ncells;
  for (int k = 0; k < 4; ++k) p.g.c[k] = a.gp[k];
  int64_t G = (a.ncells * K::NS + 255) / 256;
  if (G > 4096) G = 4096;
  if (G > a.n_partial) return (int)hipErrorInvalidValue;
  *a.n_partial_used = G;
  hipLaunchKernelGGL(k_lam<K>, dim3((unsigned)G), dim3(256), 0, a.stream, p);
  return (int)hipGetLastError();
}

template <class K>
Launchers make_fwd_launchers() {
  Launchers L;
  L.predict = &launch_predict<K>;
  L.correct = &launch_correct<K>;
  L.wave_speed = &launch_wave_speed<K>;
  L.fused = &launch_fused<K>;
  L.trace_bytes_per_cell = K::TRACE_ELEMS * (int64_t)sizeof(typename K::Real);
  L.qdofs_per_cell = (int64_t)K::NS * K::M;
  L.adj_pf_per_cell = (int64_t)2 * K::D * K::NPAR;
  L.st_face_per_cell = K::ST ? (int64_t)K::D * K::NF * K::M : 0;
  return L;
}

}  // namespace adg
