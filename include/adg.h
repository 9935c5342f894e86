/*
 * adg.h -- C ABI of the MI355X (gfx950) ADER-DG step library, libadg.so.
 *
 * One explicit ADER-DG time step on a uniform periodic Cartesian grid, as
 * defined in Charrier & Weinzierl, "Stop talking to me -- a
 * communication-avoiding ADER-DG realisation" (arXiv:1801.08682):
 *   Sec. 3, Eq. (5)/(6):  Q(T + dT) = (id + (integrateVolume + integrateFace
 *                         o solveRiemann o extrapolate) o predict) Q(T),
 * with predict evaluated once per cell (Sec. 4, Constraint 1) and only the
 * face hull of the space-time predictor kept (Sec. 4, Theorem 1).
 *
 * Conventions for every entry point
 * ---------------------------------
 *  - Every argument named d_* is a DEVICE pointer owned by the caller; the
 *    library never allocates or frees device memory after adg_init and never
 *    frees caller memory.  Device buffers must be 16-byte aligned.
 *  - Layouts (float64, contiguous):
 *      Q[cell][node][var]   cell = ix + nx*(iy + ny*iz), node = kx + n*(ky + n*kz)
 *                           with n = order + 1 Gauss-Legendre points per axis,
 *                           var innermost (m variables).
 *      params[cell][k]      per-cell material: acoustics (c), elasticity
 *                           (rho, lambda, mu); none for advection and Euler.
 *  - Calls are asynchronous: they enqueue kernels on the stream given to
 *    adg_init and return.  Numerical failures (non-finite values, rho <= 0 or
 *    p <= 0 for Euler) surface only through the device flag of adg_step.
 *  - A context is not thread-safe: one context per stream.  Calls that overlap
 *    on the same context race on its workspace.
 *  - Errors: a status code is returned; no exceptions or aborts cross the ABI.
 *    ADG_ERR_INVALID_ARG  null required pointer, misaligned buffer, bad
 *                         dimension/order/cell count, non-uniform h, bad PDE;
 *    ADG_ERR_UNSUPPORTED  valid combination of (dim, order, pde, precision)
 *                         that is not compiled into this library;
 *    ADG_ERR_WORKSPACE    workspace smaller than adg_query reported;
 *    ADG_ERR_DEVICE       a HIP launch or runtime error; adg_last_error()
 *                         gives the message.
 */
#ifndef ADG_H_
#define ADG_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  ADG_OK = 0,
  ADG_ERR_INVALID_ARG = 1,
  ADG_ERR_UNSUPPORTED = 2,
  ADG_ERR_DEVICE = 3,
  ADG_ERR_WORKSPACE = 4
} adg_status;

/* PDE of Eq. (1) with B_i = 0, S = 0 (Sec. 3); m = number of variables.
 *  ADVECTION  m = 1, pde_param = velocity (a_1..a_d)
 *  EULER      m = d + 2, Q = (rho, j, E), pde_param[0] = gamma (Sec. 7)
 *  ELASTIC    m = d + 6 (3D) / d + 3 (2D), Q = (v, Voigt stresses),
 *             params per cell (rho, lambda, mu)
 *  ACOUSTIC   m = d + 1, Q = (p, u), params per cell (c) */
typedef enum { ADG_ADVECTION = 0, ADG_EULER = 1, ADG_ELASTIC = 2, ADG_ACOUSTIC = 3 } adg_pde;

/* Arithmetic of the predictor (predict + extrapolate).  The volume
 * integration, Riemann solve, face integration and update always run in
 * float64.  FP32: float Picard iteration and float face traces.  BF16: as
 * FP32, but every pencil contraction with D of the Picard iteration takes
 * bfloat16 inputs (the flux differences to the pencil's reference flux,
 * rounded to nearest even; D as the pair Dh + Dl of two bfloat16 values) and
 * accumulates in float32 on the matrix cores (v_mfma_f32_16x16x32_bf16);
 * compiled for 3D Euler N = 3, 4, 7, 3D elasticity N = 5 and 3D acoustics
 * N = 3 (other combinations return ADG_ERR_UNSUPPORTED). */
typedef enum { ADG_FP64 = 0, ADG_FP32 = 1, ADG_BF16 = 2 } adg_precision;

typedef struct {
  int32_t dim;            /* d in {2, 3} */
  int32_t order;          /* N (the paper's p); n = N + 1 nodes per axis */
  int32_t n_cells[3];     /* periodic grid; n_cells[2] ignored when dim == 2 */
  double length[3];       /* domain edge lengths; h = length[i]/n_cells[i] must agree */
  int32_t pde;            /* adg_pde */
  double pde_param[4];    /* see adg_pde */
  int32_t picard_iters;   /* R; 0 selects N + 1 */
  int32_t precision;      /* adg_precision */
  int32_t adjoint;        /* nonzero: reserve workspace for adg_step_adjoint (FP64 only) */
  int32_t fused;          /* nonzero: reserve workspace for adg_run_fused */
  int32_t spacetime_traces; /* nonzero: the hull keeps q and F.n at every time node and the
                               Riemann problems are solved per time node (Table 1's
                               extrapolate and solveRiemann cardinalities), F* integrated in
                               time; with the FP64 or FP32 predictor (the hull in that
                               precision), every instantiated order; not with ADG_BF16, no
                               adjoint.  0: time-integrated traces (one value per face node) */
} adg_config;

typedef struct adg_ctx adg_ctx;

/* Sizes for a configuration; host-only, needs no GPU.
 *   dofs_per_cell   = m (N+1)^d   (Sec. 3: m (p+1)^d coefficients per cell)
 *   params_per_cell = per-cell material count (0, 1 or 3)
 *   workspace_bytes = device workspace the caller must pass to adg_init: the
 *                     face hull (Theorem 1; Table 1 task extrapolate: one time
 *                     value per face node, or N+1 with cfg->spacetime_traces)
 *                     plus reduction scratch; with cfg->spacetime_traces also
 *                     the time-integrated Rusanov fluxes of every cell's d
 *                     lower faces (the corrector's first pass); with
 *                     cfg->adjoint also the
 *                     hull's bars, per-block scratch of the Picard iterates
 *                     (at most 2048 blocks, at most 2 GiB) and one material
 *                     bar slot per cell face; with cfg->fused a
 *                     second Q~ buffer, a second hull and 256 bytes of time
 *                     step state.
 * Any output pointer may be NULL.  Returns INVALID_ARG / UNSUPPORTED as above. */
adg_status adg_query(const adg_config* cfg, int64_t* dofs_per_cell, int64_t* params_per_cell,
                     int64_t* workspace_bytes);

/* Create a context bound to `stream` (a hipStream_t; NULL = default stream)
 * and to the caller-owned workspace d_workspace of workspace_bytes bytes.
 * Builds the 1D Gauss-Legendre operators on the host.  *out receives the
 * context (host memory owned by the library; free with adg_destroy). */
adg_status adg_init(const adg_config* cfg, void* d_workspace, int64_t workspace_bytes, void* stream,
                    adg_ctx** out);

/* STP step (Sec. 3 "ADER-DG step 1", Eq. (3); Table 1 predict + extrapolate)
 * with integrateVolume brought forward (Sec. 5, Technique 1):
 * for every cell, Picard-iterate the space-time predictor with time step
 * *d_dt, write the time-integrated face traces into the workspace and
 * overwrite Q in place with Q~ = Q + dt * (volume term of Eq. (2)).
 * d_params may be NULL when the PDE has no per-cell parameters. */
adg_status adg_predict(adg_ctx* ctx, double* d_Q, const double* d_params, const double* d_dt);

/* Riemann + Corrector (Sec. 3 "ADER-DG steps 2 and 3"; Eq. (4) Rusanov;
 * Table 1 solveRiemann, integrateFace, update, calcTimeStep): for every cell
 * solve the Rusanov problems of its 2d faces from the traces written by
 * adg_predict, add the face term of Eq. (2) to Q~ in place, and record the
 * per-block maximum wave speed of the new state for adg_cfl_dt.
 * d_flag (nullable) is OR-ed with 1 on a non-finite state and 2 on a
 * non-physical one (or a face trace whose wave speed is not a real number);
 * the caller zeroes it. */
adg_status adg_correct(adg_ctx* ctx, double* d_Q, const double* d_params, const double* d_dt,
                       int32_t* d_flag);

/* One full time step, Alg. 1 (left) without the time-step update:
 * adg_predict followed by adg_correct.  Q(T) -> Q(T + dt) in place. */
adg_status adg_step(adg_ctx* ctx, double* d_Q, const double* d_params, const double* d_dt,
                    int32_t* d_flag);

/* Record the per-block maximum directional wave speed of Q (as adg_correct
 * does for the new state), e.g. before the first step. */
adg_status adg_wave_speed(adg_ctx* ctx, const double* d_Q, const double* d_params);

/* calcTimeStep and the global reduction (Sec. 3 "Time stepping"; Alg. 1):
 * reduce the per-block maxima recorded by the last adg_correct or
 * adg_wave_speed into *d_lambda_max (nullable) and set, on the device,
 * *d_dt = cfl * h / (d (2N + 1) lambda_max).  No host synchronisation. */
adg_status adg_cfl_dt(adg_ctx* ctx, double cfl, double* d_lambda_max, double* d_dt);

/* Shifted, fused and optimistic time stepping (Sec. 5, Techniques 3-5;
 * Alg. 2): advance Q by nsteps steps with one sweep per step.  A sweep runs,
 * per cell, the Riemann solves and corrector of step k (Delta T_old) and at
 * once the predictor of step k+1 on the new state (Delta T_new), so Q is read
 * and written once per step.  The admissible dt of the new states,
 *   dt_adm = cfl * h / (d (2N+1) lambda_max),
 * is known only after the sweep; if dt_adm < Delta T_new the sweep's
 * predictors are rerun with c_dt * dt_adm (on the device, no host
 * synchronisation).  Then Delta T_old <- Delta T_new and Delta T_new <-
 * (Delta T_old + c_dt dt_adm) / 2 (creeping != 0) or c_dt dt_adm.  The first
 * predictor uses c_dt * dt_adm(Q(T)).  The paper uses c_dt = 0.99; c_dt > 1
 * forces a rerun after every sweep.
 *   d_Q       in: Q(T); out: Q after nsteps steps (also used as a ping-pong
 *             buffer during the run);
 *   d_dt_used (nullable) out: the nsteps time steps taken, in order;
 *   d_reruns  (nullable) out: number of predictor reruns (int32);
 *   d_flag    (nullable) as in adg_correct.
 * Needs a context created with cfg->fused != 0 (else ADG_ERR_WORKSPACE);
 * nsteps >= 1, cfl > 0, c_dt > 0 (else ADG_ERR_INVALID_ARG).  Overwrites the
 * hull and the per-block maxima of the workspace. */
adg_status adg_run_fused(adg_ctx* ctx, double* d_Q, const double* d_params, int32_t nsteps,
                         double cfl, double c_dt, int32_t creeping, double* d_dt_used,
                         int32_t* d_reruns, int32_t* d_flag);

/* adg_run_fused in three parts, for callers that drive the sweeps:
 * adg_fused_begin (dt from Q(T), predictor of step 1; d_dt_used holds at most
 * dt_capacity steps, later ones are not recorded), then one adg_fused_sweep
 * per further step, then adg_fused_end (corrector of the last step into the
 * d_Q given to begin).  Arguments and errors as for adg_run_fused; sweep and
 * end without a begun run return ADG_ERR_INVALID_ARG.  Between begin and end
 * d_Q holds an intermediate (a predicted Q~), not a state. */
adg_status adg_fused_begin(adg_ctx* ctx, double* d_Q, const double* d_params, double cfl,
                           double c_dt, int32_t creeping, double* d_dt_used, int32_t dt_capacity,
                           int32_t* d_reruns, int32_t* d_flag);
adg_status adg_fused_sweep(adg_ctx* ctx);
adg_status adg_fused_end(adg_ctx* ctx);

/* Finite-volume subcell patches of the limiter (Sec. 3, "Finite Volume
 * limiter"; App. A, Corollary 8).  Every cell carries S^d subcells,
 * S = 2N + 1, as P[cell][subcell][var] (float64; subcells lexicographic with
 * the x index fastest, var innermost: S^d m values per cell).  Each call
 * reads d_in/d_P and writes the other buffer (distinct, caller-owned,
 * 16-byte aligned); contexts with precision ADG_FP64 and time-integrated
 * traces only (else ADG_ERR_UNSUPPORTED).
 *
 * adg_fv_project: P = the exact average of each cell's polynomial Q over
 * each subcell (tensor product of the per-axis averages of the Lagrange
 * basis).
 * adg_fv_reconstruct: Q = the least-squares DG solution whose subcell
 * averages best match P (per axis (Pi^T Pi)^-1 Pi^T); it inverts
 * adg_fv_project on DG data.
 * adg_fv_step: one first-order finite-volume step with Rusanov fluxes on the
 * periodic subgrid of spacing h / S, i.e. ADER-DG with p = 0 there (the
 * predictor is the identity, the face traces are the subcells' own states
 * and fluxes, Corollary 8): d_Pout = d_P - (dt S / h) sum_i (F*_{i,+} -
 * F*_{i,-}), F* = (f_L + f_R)/2 - s (P_R - P_L)/2 with s = max(lambda_L,
 * lambda_R) per face; a subcell takes its cell's material.  Records the
 * per-block maxima of the new state's wave speeds, so adg_cfl_dt then gives
 * cfl (h/S) / (d lambda_max), the subgrid's admissible step (h/S is exactly
 * the h / (2N + 1) of the DG step's formula).  d_flag as in adg_correct. */
adg_status adg_fv_project(adg_ctx* ctx, const double* d_Q, double* d_P);
adg_status adg_fv_reconstruct(adg_ctx* ctx, const double* d_P, double* d_Q);
adg_status adg_fv_step(adg_ctx* ctx, const double* d_P, double* d_Pout, const double* d_params,
                       const double* d_dt, int32_t* d_flag);

/* Reverse mode of one adg_step with dt held fixed (the discrete adjoint of
 * Eq. (5)/(6) including the Picard iterations and the Rusanov maximum; the
 * maximum passes its derivative to the first maximal face node, left state
 * before right):
 *   d_Qbar (in)  dJ/dQ(T + dt), (out) dJ/dQ(T), in place;
 *   d_params_bar (nullable) += dJ/dparams, same layout as params.
 * d_Qn is Q(T) and is not modified.  Needs a context created with
 * cfg->adjoint != 0 and precision ADG_FP64 (else ADG_ERR_WORKSPACE /
 * ADG_ERR_UNSUPPORTED).  Overwrites the face hull of the workspace. */
adg_status adg_step_adjoint(adg_ctx* ctx, const double* d_Qn, const double* d_params,
                            const double* d_dt, double* d_Qbar, double* d_params_bar);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): adg_step
 * (predict + correct, the same kernels and results) with the face hull and the
 * per-block maxima in a static device array of the library instead of a
 * caller workspace.  The array holds at most 32 MiB (33554432 bytes) per GPU
 * and stays allocated on every GPU the library ran on until the process ends.
 *   ctx           created by adg_init(cfg, NULL, 0, stream, &ctx): a context
 *                 without workspace; adg_init looks up the array's address on
 *                 the current device and returns ADG_ERR_WORKSPACE when
 *                 adg_query's workspace_bytes for cfg exceeds 32 MiB, and
 *                 ADG_ERR_INVALID_ARG when cfg->adjoint or cfg->fused is set;
 *   d_Q, d_params, d_dt, d_flag   as for adg_step;
 *   d_lambda_max  (nullable) out: the largest directional wave speed of the
 *                 new state (the input of calcTimeStep).
 * Calls no hipMalloc, hipFree or other allocating routine.  Every call on a
 * GPU uses that GPU's one array: calls that overlap on one GPU (other
 * streams, other threads, other contexts) race on it.  The array keeps the
 * last call's contents; every value a call reads was written by the same
 * call.  On a context without workspace every other stepping entry point
 * returns ADG_ERR_WORKSPACE, and adg_step_noalloc on a context with a
 * workspace does too. */
adg_status adg_step_noalloc(adg_ctx* ctx, double* d_Q, const double* d_params, const double* d_dt,
                            int32_t* d_flag, double* d_lambda_max);

/* Free a context (host memory only). */
adg_status adg_destroy(adg_ctx* ctx);

/* Last error message of a context ("" if none); ctx may be NULL for errors of
 * adg_query/adg_init.  The string is valid until the next call. */
const char* adg_last_error(const adg_ctx* ctx);

/* Library version, (major << 16) | minor. */
int32_t adg_version(void);

#ifdef __cplusplus
}
#endif

#endif /* ADG_H_ */
