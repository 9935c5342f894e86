// Device-side fluxes F_I(Q) and directional wave speeds for the four PDEs.
//
// Eq. (1) of the paper without non-conservative products, sources and point
// sources (Sec. 3 neglects them):  dQ/dt + sum_i d/dx_i F_i(Q) = 0.
// Euler is the paper's benchmark PDE (Sec. 7): Q = (rho, j, E),
// F_i = (j_i, j_i j / rho + p e_i, j_i (E + p) / rho),
// p = (gamma - 1)(E - |j|^2 / (2 rho)).
//
// Conventions shared by every PDE struct:
//   M, NPAR, LINEAR        number of variables, per-cell parameters, linearity
//   G<T>                   global constants in the working precision
//   CP<T>                  per-cell constants derived from the cell parameters
//   flux<I>(q, F, g, cp)   F = F_I(q), all M components
//   speed<I>(q, g, cp)     largest |eigenvalue| of dF_I/dQ at q
//   admissible(q, g, cp)   physical-state test used for the error flag
#pragma once

#include <hip/hip_runtime.h>

namespace adg {

template <class T> struct Gconst { T c[4]; };

// 1/x from the hardware reciprocal refined by Newton steps (double: two
// steps, within a few ulp of the correctly rounded quotient).
__device__ __forceinline__ double rcp(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}
__device__ __forceinline__ float rcp(float x) {
  float r = __builtin_amdgcn_rcpf(x);
  return fmaf(r, fmaf(-x, r, 1.0f), r);
}

// Publish form: the predictor's node threads hand the pencil threads
// w = pub(q) instead of q, and the pencils evaluate F_I = flux_pub<I>(w).
// Euler publishes the primitive state (rho, u, p), so the d fluxes of a
// space-time node share one division; the linear PDEs publish q itself.
template <int D>
struct Advection {
  static constexpr int M = 1, NPAR = 0;
  static constexpr bool LINEAR = true;
  template <class T> struct CP { };
  template <class T> __device__ static inline CP<T> cell(const double*) { return {}; }
  template <int I, class T>
  __device__ static inline void flux(const T* q, T* F, const Gconst<T>& g, const CP<T>&) {
    F[0] = g.c[I] * q[0];
  }
  template <class T>
  __device__ static inline void pub(const T* q, T* w, const Gconst<T>&) { w[0] = q[0]; }
  template <int I, class T>
  __device__ static inline void flux_pub(const T* w, T* F, const Gconst<T>& g, const CP<T>& cp) {
    flux<I>(w, F, g, cp);
  }
  template <int I, class T>
  __device__ static inline T speed(const T*, const Gconst<T>& g, const CP<T>&) {
    return fabs(g.c[I]);
  }
  template <class T>
  __device__ static inline bool admissible(const T* q, const Gconst<T>&, const CP<T>&) {
    return isfinite(q[0]);
  }
  // Reverse mode: qb += (dF_I/dq)^T Fb ; pb += (dF_I/dpar)^T Fb
  template <int I>
  __device__ static inline void flux_adj(const double*, const double* Fb, double* qb, double*,
                                         const Gconst<double>& g, const CP<double>&) {
    qb[0] += g.c[I] * Fb[0];
  }
  // qb += sb dspeed_I/dq ; pb += sb dspeed_I/dpar
  template <int I>
  __device__ static inline void speed_adj(const double*, double, double*, double*,
                                          const Gconst<double>&, const CP<double>&) {}
};

// g.c[0] = gamma, g.c[1] = gamma - 1
template <int D>
struct Euler {
  static constexpr int M = D + 2, NPAR = 0;
  static constexpr bool LINEAR = false;
  template <class T> struct CP { };
  template <class T> __device__ static inline CP<T> cell(const double*) { return {}; }
  template <class T>
  __device__ static inline T pressure(const T* q, T ir, const Gconst<T>& g) {
    T jj = q[1] * q[1];
#pragma unroll
    for (int k = 1; k < D; ++k) jj += q[1 + k] * q[1 + k];
    return g.c[1] * (q[D + 1] - T(0.5) * jj * ir);
  }
  // g.c = (gamma, gamma - 1, gamma / (gamma - 1))
  template <class T>
  __device__ static inline void pub(const T* q, T* w, const Gconst<T>& g) {
    const T ir = rcp(q[0]);
    w[0] = q[0];
#pragma unroll
    for (int k = 0; k < D; ++k) w[1 + k] = q[1 + k] * ir;
    w[D + 1] = pressure(q, ir, g);
  }
  // F_I from (rho, u, p): rho u_I, rho u_I u + p e_I, u_I (E + p) with
  // E + p = gamma/(gamma-1) p + rho |u|^2 / 2.
  template <int I, class T>
  __device__ static inline void flux_pub(const T* w, T* F, const Gconst<T>& g, const CP<T>&) {
    const T m = w[0] * w[1 + I];
    T uu = w[1] * w[1];
#pragma unroll
    for (int k = 1; k < D; ++k) uu = fma(w[1 + k], w[1 + k], uu);
    F[0] = m;
#pragma unroll
    for (int k = 0; k < D; ++k) F[1 + k] = m * w[1 + k];
    F[1 + I] += w[D + 1];
    F[D + 1] = w[1 + I] * fma(T(0.5) * w[0], uu, g.c[2] * w[D + 1]);
  }
  template <int I, class T>
  __device__ static inline void flux(const T* q, T* F, const Gconst<T>& g, const CP<T>&) {
    const T ir = rcp(q[0]);
    const T p = pressure(q, ir, g);
    const T ui = q[1 + I] * ir;
    F[0] = q[1 + I];
#pragma unroll
    for (int k = 0; k < D; ++k) F[1 + k] = q[1 + k] * ui;
    F[1 + I] += p;
    F[D + 1] = ui * (q[D + 1] + p);
  }
  template <int I, class T>
  __device__ static inline T speed(const T* q, const Gconst<T>& g, const CP<T>&) {
    const T ir = rcp(q[0]);
    const T p = pressure(q, ir, g);
    return fabs(q[1 + I] * ir) + sqrt(g.c[0] * p * ir);
  }
  template <class T>
  __device__ static inline bool admissible(const T* q, const Gconst<T>& g, const CP<T>&) {
    bool ok = true;
#pragma unroll
    for (int v = 0; v < M; ++v) ok = ok && isfinite(q[v]);
    if (!ok) return false;
    const T ir = rcp(q[0]);
    return q[0] > T(0) && pressure(q, ir, g) > T(0);
  }
  // Reverse mode of flux through ir = 1/rho, u_I = j_I ir,
  // p = (gamma-1)(E - |j|^2 ir / 2).
  template <int I>
  __device__ static inline void flux_adj(const double* q, const double* Fb, double* qb, double*,
                                         const Gconst<double>& g, const CP<double>&) {
    const double ir = 1.0 / q[0];
    const double p = pressure(q, ir, g);
    const double uI = q[1 + I] * ir;
    double uIb = 0.0, pb = 0.0, irb = 0.0;
    qb[1 + I] += Fb[0];
#pragma unroll
    for (int k = 0; k < D; ++k) {
      qb[1 + k] += Fb[1 + k] * uI;
      uIb += Fb[1 + k] * q[1 + k];
    }
    pb += Fb[1 + I];
    uIb += Fb[D + 1] * (q[D + 1] + p);
    qb[D + 1] += Fb[D + 1] * uI;
    pb += Fb[D + 1] * uI;
    qb[1 + I] += uIb * ir;
    irb += uIb * q[1 + I];
    double jj = 0.0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
      jj += q[1 + k] * q[1 + k];
      qb[1 + k] += -g.c[1] * pb * q[1 + k] * ir;
    }
    qb[D + 1] += g.c[1] * pb;
    irb += -g.c[1] * pb * 0.5 * jj;
    qb[0] += -irb * ir * ir;
  }
  // Reverse mode of speed_I = |u_I| + sqrt(gamma p ir) (d|x|/dx = 0 at 0).
  template <int I>
  __device__ static inline void speed_adj(const double* q, double sb, double* qb, double*,
                                          const Gconst<double>& g, const CP<double>&) {
    const double ir = 1.0 / q[0];
    const double p = pressure(q, ir, g);
    const double uI = q[1 + I] * ir;
    const double cs = sqrt(g.c[0] * p * ir);
    const double sg = uI > 0.0 ? 1.0 : (uI < 0.0 ? -1.0 : 0.0);
    double uIb = sb * sg;
    const double xb = sb / (2.0 * cs);          // bar of gamma p ir
    double pb = xb * g.c[0] * ir;
    double irb = xb * g.c[0] * p;
    qb[1 + I] += uIb * ir;
    irb += uIb * q[1 + I];
    double jj = 0.0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
      jj += q[1 + k] * q[1 + k];
      qb[1 + k] += -g.c[1] * pb * q[1 + k] * ir;
    }
    qb[D + 1] += g.c[1] * pb;
    irb += -g.c[1] * pb * 0.5 * jj;
    qb[0] += -irb * ir * ir;
  }
};

// Per cell: par[0] = sound speed c (rho_0 = 1, bulk modulus c^2).
// Q = (p, u_1..u_D), F_i = (c^2 u_i, p e_i).
template <int D>
struct Acoustic {
  static constexpr int M = D + 1, NPAR = 1;
  static constexpr bool LINEAR = true;
  template <class T> struct CP { T c, K; };
  template <class T> __device__ static inline CP<T> cell(const double* par) {
    const double c = par[0];
    return {T(c), T(c * c)};
  }
  template <int I, class T>
  __device__ static inline void flux(const T* q, T* F, const Gconst<T>&, const CP<T>& cp) {
    F[0] = cp.K * q[1 + I];
#pragma unroll
    for (int k = 0; k < D; ++k) F[1 + k] = (k == I) ? q[0] : T(0);
  }
  template <class T>
  __device__ static inline void pub(const T* q, T* w, const Gconst<T>&) {
#pragma unroll
    for (int v = 0; v < M; ++v) w[v] = q[v];
  }
  template <int I, class T>
  __device__ static inline void flux_pub(const T* w, T* F, const Gconst<T>& g, const CP<T>& cp) {
    flux<I>(w, F, g, cp);
  }
  template <int I, class T>
  __device__ static inline T speed(const T*, const Gconst<T>&, const CP<T>& cp) { return cp.c; }
  template <class T>
  __device__ static inline bool admissible(const T* q, const Gconst<T>&, const CP<T>&) {
    bool ok = true;
#pragma unroll
    for (int v = 0; v < M; ++v) ok = ok && isfinite(q[v]);
    return ok;
  }
  // F_I = (c^2 u_I, p e_I): pb[0] is the bar of the sound speed c.
  template <int I>
  __device__ static inline void flux_adj(const double* q, const double* Fb, double* qb, double* pb,
                                         const Gconst<double>&, const CP<double>& cp) {
    qb[1 + I] += cp.K * Fb[0];
    qb[0] += Fb[1 + I];
    pb[0] += 2.0 * cp.c * q[1 + I] * Fb[0];
  }
  template <int I>
  __device__ static inline void speed_adj(const double*, double sb, double*, double* pb,
                                          const Gconst<double>&, const CP<double>&) {
    pb[0] += sb;
  }
};

// Per cell: par = (rho, lambda, mu).  Velocity-stress form, stresses in
// Voigt order (11,22,33,12,23,13) in 3D and (11,22,12) in 2D.
// F_i(v_k) = -sigma_ik / rho,
// F_i(sigma_kl) = -(lambda delta_kl v_i + mu (delta_ik v_l + delta_il v_k)).
template <int D>
struct Elastic {
  static constexpr int NS_ = (D == 3) ? 6 : 3;
  static constexpr int M = D + NS_, NPAR = 3;
  static constexpr bool LINEAR = true;
  template <class T> struct CP { T irho, lam, mu, cp; };
  template <class T> __device__ static inline CP<T> cell(const double* par) {
    const double rho = par[0], lam = par[1], mu = par[2];
    return {T(1.0 / rho), T(lam), T(mu), T(sqrt((lam + 2.0 * mu) / rho))};
  }
  // Voigt slot of the symmetric pair (k, l)
  __host__ __device__ static constexpr int slot(int k, int l) {
    return (D == 3)
               ? ((k == l) ? k : ((k + l == 1) ? 3 : ((k + l == 3) ? 4 : 5)))
               : ((k == l) ? k : 2);
  }
  __host__ __device__ static constexpr int vk(int s) {   // first index of slot s
    return (D == 3) ? (s < 3 ? s : (s == 3 ? 0 : (s == 4 ? 1 : 0)))
                    : (s < 2 ? s : 0);
  }
  __host__ __device__ static constexpr int vl(int s) {   // second index of slot s
    return (D == 3) ? (s < 3 ? s : (s == 3 ? 1 : (s == 4 ? 2 : 2)))
                    : (s < 2 ? s : 1);
  }
  template <int I, class T>
  __device__ static inline void flux(const T* q, T* F, const Gconst<T>&, const CP<T>& cp) {
#pragma unroll
    for (int k = 0; k < D; ++k) F[k] = -q[D + slot(I, k)] * cp.irho;
#pragma unroll
    for (int s = 0; s < NS_; ++s) {
      const int k = vk(s), l = vl(s);
      T t = T(0);
      if (I == k) t += cp.mu * q[l];
      if (I == l) t += cp.mu * q[k];
      if (k == l) t += cp.lam * q[I];
      F[D + s] = -t;
    }
  }
  template <class T>
  __device__ static inline void pub(const T* q, T* w, const Gconst<T>&) {
#pragma unroll
    for (int v = 0; v < M; ++v) w[v] = q[v];
  }
  template <int I, class T>
  __device__ static inline void flux_pub(const T* w, T* F, const Gconst<T>& g, const CP<T>& cp) {
    flux<I>(w, F, g, cp);
  }
  template <int I, class T>
  __device__ static inline T speed(const T*, const Gconst<T>&, const CP<T>& cp) { return cp.cp; }
  template <class T>
  __device__ static inline bool admissible(const T* q, const Gconst<T>&, const CP<T>&) {
    bool ok = true;
#pragma unroll
    for (int v = 0; v < M; ++v) ok = ok && isfinite(q[v]);
    return ok;
  }
  // pb = bars of (rho, lambda, mu).
  template <int I>
  __device__ static inline void flux_adj(const double* q, const double* Fb, double* qb, double* pb,
                                         const Gconst<double>&, const CP<double>& cp) {
#pragma unroll
    for (int k = 0; k < D; ++k) {
      qb[D + slot(I, k)] += -Fb[k] * cp.irho;
      pb[0] += Fb[k] * q[D + slot(I, k)] * cp.irho * cp.irho;
    }
#pragma unroll
    for (int s = 0; s < NS_; ++s) {
      const int k = vk(s), l = vl(s);
      const double fb = -Fb[D + s];
      if (I == k) { qb[l] += cp.mu * fb; pb[2] += q[l] * fb; }
      if (I == l) { qb[k] += cp.mu * fb; pb[2] += q[k] * fb; }
      if (k == l) { qb[I] += cp.lam * fb; pb[1] += q[I] * fb; }
    }
  }
  // speed = sqrt((lambda + 2 mu) / rho)
  template <int I>
  __device__ static inline void speed_adj(const double*, double sb, double*, double* pb,
                                          const Gconst<double>&, const CP<double>& cp) {
    const double x = 0.5 * sb / cp.cp;            // bar of (lambda + 2 mu) / rho
    pb[1] += x * cp.irho;
    pb[2] += 2.0 * x * cp.irho;
    pb[0] += -x * cp.cp * cp.cp * cp.irho;
  }
};

}  // namespace adg
