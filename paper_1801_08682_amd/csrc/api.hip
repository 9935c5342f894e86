// C ABI of libadg.so (declared in include/adg.h): validation, workspace
// layout, the 1D operator tables and kernel dispatch.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>

#include "../../include/adg.h"
#include "common.hpp"
#include "kernels_fwd.hpp"

namespace {

thread_local std::string g_err;

struct Layout {
  int64_t trace_off = 0, trace_bytes = 0;
  int64_t partial_off = 0, partial_count = 0;
  int64_t tb_off = 0, slots_off = 0, nslots = 0, pf_off = 0;
  int64_t stf_off = -1;
  int64_t q2_off = 0, tr2_off = 0, fz_off = 0;   // fused stepping: second Q~, second hull, dt state
  int64_t total = 0;
};

// Per-block Picard scratch of the adjoint: at most 2048 blocks and 2 GiB.
int64_t adjoint_slots(int64_t cells, int64_t slot_bytes) {
  int64_t s = cells < 2048 ? cells : 2048;
  const int64_t cap = (int64_t(2) << 30) / (slot_bytes > 0 ? slot_bytes : 1);
  if (s > cap) s = cap > 1 ? cap : 1;
  return s;
}

int64_t align256(int64_t x) { return (x + 255) & ~int64_t(255); }

int n_vars(int pde, int dim) {
  switch (pde) {
    case ADG_ADVECTION: return 1;
    case ADG_EULER: return dim + 2;
    case ADG_ACOUSTIC: return dim + 1;
    case ADG_ELASTIC: return dim + (dim == 3 ? 6 : 3);
  }
  return 0;
}

int n_params(int pde) {
  return pde == ADG_ACOUSTIC ? 1 : (pde == ADG_ELASTIC ? 3 : 0);
}

adg_status validate(const adg_config* c, std::string* msg) {
  if (!c) { *msg = "config is NULL"; return ADG_ERR_INVALID_ARG; }
  if (c->dim != 2 && c->dim != 3) { *msg = "dim must be 2 or 3"; return ADG_ERR_INVALID_ARG; }
  if (c->order < 0 || c->order > 15) { *msg = "order must be in [0, 15]"; return ADG_ERR_INVALID_ARG; }
  if (c->pde < 0 || c->pde > 3) { *msg = "unknown pde"; return ADG_ERR_INVALID_ARG; }
  if (c->precision < 0 || c->precision > 2) { *msg = "unknown precision"; return ADG_ERR_INVALID_ARG; }
  if (c->adjoint != 0 && c->precision != ADG_FP64) {
    *msg = "the adjoint needs precision ADG_FP64";
    return ADG_ERR_UNSUPPORTED;
  }
  if (c->picard_iters < 0 || c->picard_iters > 1000) {
    *msg = "picard_iters must be in [0, 1000]";
    return ADG_ERR_INVALID_ARG;
  }
  double h0 = 0.0;
  int64_t cells = 1;
  for (int i = 0; i < c->dim; ++i) {
    if (c->n_cells[i] < 1) { *msg = "n_cells must be >= 1"; return ADG_ERR_INVALID_ARG; }
    if (!(c->length[i] > 0.0) || !std::isfinite(c->length[i])) {
      *msg = "length must be positive";
      return ADG_ERR_INVALID_ARG;
    }
    const double h = c->length[i] / c->n_cells[i];
    if (i == 0) h0 = h;
    else if (std::fabs(h - h0) > 1e-12 * h0) { *msg = "cell width must be uniform"; return ADG_ERR_INVALID_ARG; }
    cells *= c->n_cells[i];
  }
  if (cells > (int64_t(1) << 31)) { *msg = "too many cells"; return ADG_ERR_INVALID_ARG; }
  if (c->pde == ADG_EULER) {
    const double g = c->pde_param[0] == 0.0 ? 1.4 : c->pde_param[0];
    if (!(g > 1.0)) { *msg = "Euler needs gamma > 1"; return ADG_ERR_INVALID_ARG; }
  }
  return ADG_OK;
}

const adg::Launchers* find(const adg_config* c) {
  switch (c->pde) {
    case ADG_ADVECTION: return adg::find_advection(c->dim, c->order, c->precision, c->spacetime_traces != 0);
    case ADG_EULER: return adg::find_euler(c->dim, c->order, c->precision, c->spacetime_traces != 0);
    case ADG_ACOUSTIC: return adg::find_acoustic(c->dim, c->order, c->precision, c->spacetime_traces != 0);
    case ADG_ELASTIC: return adg::find_elastic(c->dim, c->order, c->precision, c->spacetime_traces != 0);
  }
  return nullptr;
}

int64_t n_cells_of(const adg_config* c) {
  int64_t k = 1;
  for (int i = 0; i < c->dim; ++i) k *= c->n_cells[i];
  return k;
}

Layout layout_of(const adg_config* c, const adg::Launchers* L) {
  Layout l;
  const int64_t cells = n_cells_of(c);
  l.trace_off = 0;
  l.trace_bytes = align256(cells * L->trace_bytes_per_cell);
  l.partial_off = l.trace_off + l.trace_bytes;
  // one maximum per corrector workgroup (padded to 8) or per reduction block
  // plus 256 slots for the first stage of the dt reduction
  l.partial_count = (cells + 64 > adg::kMaxReduceBlocks ? cells + 64 : adg::kMaxReduceBlocks) + 256;
  l.total = l.partial_off + align256(l.partial_count * 8);
  if (L->st_face_per_cell > 0) {      // space-time traces: F* of the lower faces
    l.stf_off = l.total;
    l.total = l.stf_off + align256(cells * L->st_face_per_cell * 8);
  }
  if (c->adjoint && L->adjoint) {
    const int R = c->picard_iters > 0 ? c->picard_iters : c->order + 1;
    const int64_t slot = L->adj_slot_doubles(R) * 8;
    l.tb_off = l.total;
    l.slots_off = l.tb_off + align256(cells * L->trace_bytes_per_cell);
    l.nslots = adjoint_slots(cells, slot);
    l.pf_off = l.slots_off + align256(l.nslots * slot);
    l.total = l.pf_off + align256(cells * L->adj_pf_per_cell * 8);
  }
  if (c->fused) {
    l.q2_off = l.total;
    l.tr2_off = l.q2_off + align256(cells * L->qdofs_per_cell * 8);
    l.fz_off = l.tr2_off + align256(cells * L->trace_bytes_per_cell);
    l.total = l.fz_off + 256;
  }
  return l;
}

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

// Scratch of adg_step_noalloc: the face hull and the per-block maxima of one
// step, in a file-scope device array (one copy per GPU, held until the process
// ends).  Host code never passes `scratch` itself to a kernel: its device
// address on the current GPU comes from hipGetSymbolAddress, taken once per
// device by adg_init and kept in g_scratch_ptr.
constexpr int64_t kStaticScratchBytes = int64_t(32) << 20;
constexpr int kMaxDevices = 64;
__device__ __align__(256) static double scratch[kStaticScratchBytes / 8];
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up on first use).
adg_status static_scratch(void** out, std::string* msg) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) { *msg = std::string("hipGetDevice: ") + hipGetErrorString(e); return ADG_ERR_DEVICE; }
  if (dev < 0 || dev >= kMaxDevices) { *msg = "device index out of range"; return ADG_ERR_DEVICE; }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      *msg = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
      return ADG_ERR_DEVICE;
    }
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return ADG_OK;
}

// First stage of the global maximum: 256 blocks, one maximum each.
__global__ void __launch_bounds__(256) k_max256(const double* partial, int64_t cnt, double* out) {
  __shared__ double red[4];
  double m = 0.0;
  for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k < cnt; k += 256 * 256)
    m = fmax(m, partial[k]);
  m = adg::block_max<256>(m, red);
  if (threadIdx.x == 0) out[blockIdx.x] = m;
}

__global__ void __launch_bounds__(256) k_dt(const double* partial, int64_t cnt, double coef,
                                            double* lam_out, double* dt_out) {
  __shared__ double red[4];
  double m = 0.0;
  for (int64_t k = threadIdx.x; k < cnt; k += 256) m = fmax(m, partial[k]);
  m = adg::block_max<256>(m, red);
  if (threadIdx.x == 0) {
    if (lam_out) *lam_out = m;
    if (dt_out) *dt_out = coef / m;
  }
}

// Time step state of the fused scheme (device memory, in the workspace).
struct FzState {
  double dt_corr;     // dt of the next sweep's corrector (the dt its predictors used)
  double dt_stp;      // dt of the next sweep's predictors (Delta T_new)
  double dtc_rerun;   // rerun: the corrector's dt (unchanged)
  double dts_rerun;   // rerun: the predictors' reset dt
  double lam;         // largest wave speed of the last sweep's new states
  double dt_adm;      // the admissible dt of those states
  int32_t rerun;      // 1: the last sweep's predictors must be rerun
  int32_t reruns;     // reruns so far
};

// Optimistic time step control (Sec. 5 Technique 5; Alg. 2), one block.
// dt_adm = coef / lambda_max with coef = C h / (d (2N+1)).
//  mode 0 (start, lambda of Q^0): dt_corr = dt_stp = c_dt dt_adm.
//  mode 1 (after sweep k: corrector of step k, predictors of step k+1):
//    dt_used[k-1] = dt_corr; if dt_adm < dt_stp the predictors overshot:
//    rerun them with dts_rerun = c_dt dt_adm (corrector unchanged).  Then
//    Delta T_old = dt_stp (as finally used), Delta T_new = the creeping
//    average (Delta T_old + c_dt dt_adm) / 2, or c_dt dt_adm.
//  mode 2 (before the last corrector): dt_used[k-1] = dt_corr.
__global__ void __launch_bounds__(256) k_fz_dt(const double* partial, int64_t cnt, double coef,
                                               double c_dt, int creeping, int mode, FzState* st,
                                               double* dt_used, int64_t k, int32_t* reruns_out) {
  __shared__ double red[4];
  double m = 0.0;
  if (mode != 2)
    for (int64_t i = threadIdx.x; i < cnt; i += 256) m = fmax(m, partial[i]);
  m = adg::block_max<256>(m, red);
  if (threadIdx.x != 0) return;
  if (mode == 2) {
    if (dt_used) dt_used[k - 1] = st->dt_corr;
    return;
  }
  const double adm = coef / m;
  st->lam = m;
  st->dt_adm = adm;
  if (mode == 0) {
    st->dt_corr = c_dt * adm;
    st->dt_stp = c_dt * adm;
    st->rerun = 0;
    st->reruns = 0;
  } else {
    if (dt_used) dt_used[k - 1] = st->dt_corr;
    double used = st->dt_stp;
    if (adm < used) {
      st->rerun = 1;
      st->reruns += 1;
      st->dtc_rerun = st->dt_corr;
      st->dts_rerun = c_dt * adm;
      used = c_dt * adm;
    } else {
      st->rerun = 0;
    }
    st->dt_corr = used;
    st->dt_stp = creeping ? 0.5 * (used + c_dt * adm) : c_dt * adm;
  }
  if (reruns_out) *reruns_out = st->reruns;
}

}  // namespace

struct adg_ctx {
  adg_config cfg;
  const adg::Launchers* L = nullptr;
  adg::HostTables tab;
  hipStream_t stream = nullptr;
  char* ws = nullptr;
  bool static_ws = false;       // ws is the static scratch: only adg_step_noalloc may run
  Layout lay;
  int64_t n_partial_used = 0;
  int64_t ncells = 0;
  double h = 1.0;
  int R = 1;
  double gp[4] = {0, 0, 0, 0};
  std::string err;
  struct FusedRun {             // host side of a fused run (adg_fused_begin .. end)
    bool active = false;
    double* Q = nullptr;
    const double* params = nullptr;
    int32_t* flag = nullptr;
    double* dt_used = nullptr;
    int32_t dt_capacity = 0;
    int32_t* reruns = nullptr;
    double coef = 0.0, c_dt = 1.0;
    int32_t creeping = 1;
    int cur = 1, curt = 0;      // (Q~, hull) of the step in flight
    int32_t k = 0;              // steps begun
  } fz;

  adg::LaunchArgs args() {
    adg::LaunchArgs a;
    a.traces = ws + lay.trace_off;
    a.partial = reinterpret_cast<double*>(ws + lay.partial_off);
    a.n_partial = lay.partial_count - 256;   // the last 256 slots stage the dt reduction
    a.n_partial_used = &n_partial_used;
    if (lay.stf_off >= 0) a.st_face = reinterpret_cast<double*>(ws + lay.stf_off);
    if (lay.nslots > 0) {
      a.adj_tb = reinterpret_cast<double*>(ws + lay.tb_off);
      a.adj_slots = reinterpret_cast<double*>(ws + lay.slots_off);
      a.adj_nslots = lay.nslots;
      a.adj_pf = reinterpret_cast<double*>(ws + lay.pf_off);
    }
    a.ncells = ncells;
    for (int i = 0; i < 3; ++i) {
      a.nc[i] = (i < cfg.dim) ? cfg.n_cells[i] : 1;
      int b = 1;                      // largest divisor of the axis length up to 16
      for (int d = 16; d >= 1; --d)
        if (a.nc[i] % d == 0) { b = d; break; }
      a.brick[i] = b;
    }
    a.inv_h = 1.0 / h;
    a.R = R;
    for (int k = 0; k < 4; ++k) a.gp[k] = gp[k];
    a.tab = &tab;
    a.stream = stream;
    return a;
  }
  adg_status fail(adg_status s, const std::string& m) {
    err = m;
    return s;
  }
  adg_status launched(int e, const char* what) {
    if (e != 0) {
      err = std::string(what) + ": " + hipGetErrorString((hipError_t)e);
      return ADG_ERR_DEVICE;
    }
    return ADG_OK;
  }
};

extern "C" {

int32_t adg_version(void) { return (1 << 16) | 0; }

const char* adg_last_error(const adg_ctx* ctx) { return ctx ? ctx->err.c_str() : g_err.c_str(); }

adg_status adg_query(const adg_config* cfg, int64_t* dofs_per_cell, int64_t* params_per_cell,
                     int64_t* workspace_bytes) {
  std::string msg;
  adg_status s = validate(cfg, &msg);
  if (s != ADG_OK) { g_err = msg; return s; }
  const adg::Launchers* L = find(cfg);
  if (!L) { g_err = "combination (dim, order, pde, precision) not compiled"; return ADG_ERR_UNSUPPORTED; }
  int64_t nn = 1;
  for (int i = 0; i < cfg->dim; ++i) nn *= (cfg->order + 1);
  if (dofs_per_cell) *dofs_per_cell = nn * n_vars(cfg->pde, cfg->dim);
  if (params_per_cell) *params_per_cell = n_params(cfg->pde);
  if (workspace_bytes) *workspace_bytes = layout_of(cfg, L).total;
  g_err.clear();
  return ADG_OK;
}

adg_status adg_init(const adg_config* cfg, void* d_workspace, int64_t workspace_bytes, void* stream,
                    adg_ctx** out) {
  if (!out) { g_err = "out is NULL"; return ADG_ERR_INVALID_ARG; }
  *out = nullptr;
  int64_t need = 0;
  adg_status s = adg_query(cfg, nullptr, nullptr, &need);
  if (s != ADG_OK) return s;
  void* sp = nullptr;
  const bool static_ws = !d_workspace && workspace_bytes == 0;
  if (static_ws) {
    // context for adg_step_noalloc: the library's static scratch replaces the workspace
    if (cfg->adjoint || cfg->fused) {
      g_err = "a context without workspace (adg_step_noalloc) needs adjoint = 0 and fused = 0";
      return ADG_ERR_INVALID_ARG;
    }
    if (need > kStaticScratchBytes) {
      g_err = "adg_step_noalloc: this grid needs " + std::to_string(need) +
              " bytes of scratch, the static maximum is " + std::to_string(kStaticScratchBytes);
      return ADG_ERR_WORKSPACE;
    }
    std::string msg;
    if ((s = static_scratch(&sp, &msg)) != ADG_OK) { g_err = msg; return s; }
  } else {
    if (!d_workspace) { g_err = "workspace is NULL"; return ADG_ERR_INVALID_ARG; }
    if (!aligned16(d_workspace)) { g_err = "workspace not 16-byte aligned"; return ADG_ERR_INVALID_ARG; }
    if (workspace_bytes < need) { g_err = "workspace too small"; return ADG_ERR_WORKSPACE; }
  }
  adg_ctx* c = new adg_ctx();
  c->cfg = *cfg;
  c->L = find(cfg);
  if (!adg::build_tables(cfg->order + 1, &c->tab)) {
    delete c;
    g_err = "table construction failed";
    return ADG_ERR_INVALID_ARG;
  }
  c->stream = reinterpret_cast<hipStream_t>(stream);
  c->ws = reinterpret_cast<char*>(static_ws ? sp : d_workspace);
  c->static_ws = static_ws;
  c->lay = layout_of(cfg, c->L);
  c->ncells = n_cells_of(cfg);
  c->h = cfg->length[0] / cfg->n_cells[0];
  c->R = cfg->picard_iters > 0 ? cfg->picard_iters : cfg->order + 1;
  if (cfg->pde == ADG_EULER) {
    const double g = cfg->pde_param[0] == 0.0 ? 1.4 : cfg->pde_param[0];
    c->gp[0] = g;
    c->gp[1] = g - 1.0;
    c->gp[2] = g / (g - 1.0);
  } else {
    for (int k = 0; k < 4; ++k) c->gp[k] = cfg->pde_param[k];
  }
  *out = c;
  g_err.clear();
  return ADG_OK;
}

adg_status adg_destroy(adg_ctx* ctx) {
  delete ctx;
  return ADG_OK;
}

static adg_status check_state(adg_ctx* ctx, const void* Q, const void* params, const void* dt,
                              bool noalloc = false) {
  if (!ctx) { g_err = "ctx is NULL"; return ADG_ERR_INVALID_ARG; }
  if (ctx->static_ws != noalloc)
    return ctx->fail(ADG_ERR_WORKSPACE, noalloc ? "adg_step_noalloc needs a context created without workspace"
                                                : "context has no workspace: only adg_step_noalloc runs on it");
  if (!Q || !dt) return ctx->fail(ADG_ERR_INVALID_ARG, "Q and dt are required");
  if (n_params(ctx->cfg.pde) > 0 && !params)
    return ctx->fail(ADG_ERR_INVALID_ARG, "this PDE needs per-cell params");
  if (!aligned16(Q) || (params && !aligned16(params)))
    return ctx->fail(ADG_ERR_INVALID_ARG, "device buffers must be 16-byte aligned");
  return ADG_OK;
}

adg_status adg_predict(adg_ctx* ctx, double* d_Q, const double* d_params, const double* d_dt) {
  adg_status s = check_state(ctx, d_Q, d_params, d_dt);
  if (s != ADG_OK) return s;
  adg::LaunchArgs a = ctx->args();
  a.Q = d_Q;
  a.params = d_params;
  a.dt = d_dt;
  return ctx->launched(ctx->L->predict(a), "predict");
}

adg_status adg_correct(adg_ctx* ctx, double* d_Q, const double* d_params, const double* d_dt,
                       int32_t* d_flag) {
  adg_status s = check_state(ctx, d_Q, d_params, d_dt);
  if (s != ADG_OK) return s;
  adg::LaunchArgs a = ctx->args();
  a.Q = d_Q;
  a.params = d_params;
  a.dt = d_dt;
  a.flag = d_flag;
  return ctx->launched(ctx->L->correct(a), "correct");
}

adg_status adg_step(adg_ctx* ctx, double* d_Q, const double* d_params, const double* d_dt,
                    int32_t* d_flag) {
  adg_status s = adg_predict(ctx, d_Q, d_params, d_dt);
  if (s != ADG_OK) return s;
  return adg_correct(ctx, d_Q, d_params, d_dt, d_flag);
}

adg_status adg_wave_speed(adg_ctx* ctx, const double* d_Q, const double* d_params) {
  double one = 1.0;
  adg_status s = check_state(ctx, d_Q, d_params, &one);
  if (s != ADG_OK) return s;
  adg::LaunchArgs a = ctx->args();
  a.Qc = d_Q;
  a.params = d_params;
  return ctx->launched(ctx->L->wave_speed(a), "wave_speed");
}

// Stage the recorded per-block maxima for a one-block reduction.
static void stage_partial(adg_ctx* ctx, const double** part, int64_t* cnt) {
  *part = reinterpret_cast<const double*>(ctx->ws + ctx->lay.partial_off);
  *cnt = ctx->n_partial_used;
  if (*cnt > 4096) {
    double* stage = reinterpret_cast<double*>(ctx->ws + ctx->lay.partial_off) + ctx->lay.partial_count - 256;
    hipLaunchKernelGGL(k_max256, dim3(256), dim3(256), 0, ctx->stream, *part, *cnt, stage);
    *part = stage;
    *cnt = 256;
  }
}

adg_status adg_cfl_dt(adg_ctx* ctx, double cfl, double* d_lambda_max, double* d_dt) {
  if (!ctx) { g_err = "ctx is NULL"; return ADG_ERR_INVALID_ARG; }
  if (ctx->static_ws)
    return ctx->fail(ADG_ERR_WORKSPACE, "context has no workspace: only adg_step_noalloc runs on it");
  if (!(cfl > 0.0)) return ctx->fail(ADG_ERR_INVALID_ARG, "cfl must be positive");
  if (!d_lambda_max && !d_dt) return ctx->fail(ADG_ERR_INVALID_ARG, "no output");
  if (ctx->n_partial_used <= 0)
    return ctx->fail(ADG_ERR_INVALID_ARG, "no wave speeds recorded (call adg_correct or adg_wave_speed)");
  const double coef = cfl * ctx->h / (ctx->cfg.dim * (2.0 * ctx->cfg.order + 1.0));
  const double* part = nullptr;
  int64_t cnt = 0;
  stage_partial(ctx, &part, &cnt);
  hipLaunchKernelGGL(k_dt, dim3(1), dim3(256), 0, ctx->stream, part, cnt, coef, d_lambda_max, d_dt);
  return ctx->launched((int)hipGetLastError(), "cfl_dt");
}

adg_status adg_step_noalloc(adg_ctx* ctx, double* d_Q, const double* d_params, const double* d_dt,
                            int32_t* d_flag, double* d_lambda_max) {
  adg_status s = check_state(ctx, d_Q, d_params, d_dt, true);
  if (s != ADG_OK) return s;
  if (ctx->lay.total > kStaticScratchBytes)     // adg_init checked it too
    return ctx->fail(ADG_ERR_WORKSPACE, "adg_step_noalloc: grid exceeds the static scratch");
  adg::LaunchArgs a = ctx->args();
  a.Q = d_Q;
  a.params = d_params;
  a.dt = d_dt;
  if ((s = ctx->launched(ctx->L->predict(a), "noalloc: predict")) != ADG_OK) return s;
  a.flag = d_flag;
  if ((s = ctx->launched(ctx->L->correct(a), "noalloc: correct")) != ADG_OK) return s;
  if (d_lambda_max) {
    const double* part = nullptr;
    int64_t cnt = 0;
    stage_partial(ctx, &part, &cnt);
    hipLaunchKernelGGL(k_dt, dim3(1), dim3(256), 0, ctx->stream, part, cnt, 1.0, d_lambda_max,
                       static_cast<double*>(nullptr));
    return ctx->launched((int)hipGetLastError(), "noalloc: lambda_max");
  }
  return ADG_OK;
}

static void fz_dt(adg_ctx* ctx, int mode) {
  adg_ctx::FusedRun& r = ctx->fz;
  FzState* st = reinterpret_cast<FzState*>(ctx->ws + ctx->lay.fz_off);
  const double* part = nullptr;
  int64_t cnt = 0;
  if (mode != 2) stage_partial(ctx, &part, &cnt);
  double* rec = (r.dt_used && r.k <= r.dt_capacity) ? r.dt_used : nullptr;
  hipLaunchKernelGGL(k_fz_dt, dim3(1), dim3(256), 0, ctx->stream, part, cnt, r.coef, r.c_dt,
                     r.creeping, mode, st, rec, (int64_t)r.k, r.reruns);
}

adg_status adg_fused_begin(adg_ctx* ctx, double* d_Q, const double* d_params, double cfl, double c_dt,
                           int32_t creeping, double* d_dt_used, int32_t dt_capacity,
                           int32_t* d_reruns, int32_t* d_flag) {
  double one = 1.0;
  adg_status s = check_state(ctx, d_Q, d_params, &one);
  if (s != ADG_OK) return s;
  if (!(cfl > 0.0) || !(c_dt > 0.0)) return ctx->fail(ADG_ERR_INVALID_ARG, "cfl and c_dt must be positive");
  if (ctx->lay.fz_off <= 0)
    return ctx->fail(ADG_ERR_WORKSPACE, "fused workspace not reserved (set adg_config.fused)");
  adg_ctx::FusedRun& r = ctx->fz;
  r = adg_ctx::FusedRun();
  r.Q = d_Q;
  r.params = d_params;
  r.flag = d_flag;
  r.dt_used = d_dt_used;
  r.dt_capacity = d_dt_used ? dt_capacity : 0;
  r.reruns = d_reruns;
  r.coef = cfl * ctx->h / (ctx->cfg.dim * (2.0 * ctx->cfg.order + 1.0));
  r.c_dt = c_dt;
  r.creeping = creeping;
  FzState* st = reinterpret_cast<FzState*>(ctx->ws + ctx->lay.fz_off);
  adg::LaunchArgs a = ctx->args();
  a.params = d_params;
  a.flag = d_flag;
  // dt from the speeds of Q(T), then the predictor of step 1: Q -> (Q2, hull 0)
  a.Qc = d_Q;
  if ((s = ctx->launched(ctx->L->wave_speed(a), "fused: wave_speed")) != ADG_OK) return s;
  fz_dt(ctx, 0);
  a.Q = d_Q;
  a.qin = d_Q;
  a.qout = reinterpret_cast<double*>(ctx->ws + ctx->lay.q2_off);
  a.traces = ctx->ws + ctx->lay.trace_off;
  a.dt = &st->dt_stp;
  if ((s = ctx->launched(ctx->L->predict(a), "fused: predict")) != ADG_OK) return s;
  r.cur = 1;
  r.curt = 0;
  r.k = 1;
  r.active = true;
  return ADG_OK;
}

adg_status adg_fused_sweep(adg_ctx* ctx) {
  if (!ctx) { g_err = "ctx is NULL"; return ADG_ERR_INVALID_ARG; }
  adg_ctx::FusedRun& r = ctx->fz;
  if (!r.active) return ctx->fail(ADG_ERR_INVALID_ARG, "no fused run (call adg_fused_begin)");
  FzState* st = reinterpret_cast<FzState*>(ctx->ws + ctx->lay.fz_off);
  double* X[2] = {r.Q, reinterpret_cast<double*>(ctx->ws + ctx->lay.q2_off)};
  void* T[2] = {ctx->ws + ctx->lay.trace_off, ctx->ws + ctx->lay.tr2_off};
  adg::LaunchArgs a = ctx->args();
  a.params = r.params;
  a.flag = r.flag;
  a.Q = r.Q;
  a.qin = X[r.cur];
  a.qout = X[1 - r.cur];
  a.traces = T[r.curt];
  a.traces_out = T[1 - r.curt];
  a.dt = &st->dt_corr;
  a.dt_pred = &st->dt_stp;
  adg_status s;
  if ((s = ctx->launched(ctx->L->fused(a), "fused: sweep")) != ADG_OK) return s;
  fz_dt(ctx, 1);
  a.dt = &st->dtc_rerun;
  a.dt_pred = &st->dts_rerun;
  a.run_if = &st->rerun;
  if ((s = ctx->launched(ctx->L->fused(a), "fused: rerun")) != ADG_OK) return s;
  r.cur = 1 - r.cur;
  r.curt = 1 - r.curt;
  r.k += 1;
  return ADG_OK;
}

adg_status adg_fused_end(adg_ctx* ctx) {
  if (!ctx) { g_err = "ctx is NULL"; return ADG_ERR_INVALID_ARG; }
  adg_ctx::FusedRun& r = ctx->fz;
  if (!r.active) return ctx->fail(ADG_ERR_INVALID_ARG, "no fused run (call adg_fused_begin)");
  FzState* st = reinterpret_cast<FzState*>(ctx->ws + ctx->lay.fz_off);
  double* X[2] = {r.Q, reinterpret_cast<double*>(ctx->ws + ctx->lay.q2_off)};
  void* T[2] = {ctx->ws + ctx->lay.trace_off, ctx->ws + ctx->lay.tr2_off};
  fz_dt(ctx, 2);
  adg::LaunchArgs a = ctx->args();
  a.params = r.params;
  a.flag = r.flag;
  a.Q = r.Q;
  a.qin = X[r.cur];
  a.qout = r.Q;
  a.traces = T[r.curt];
  a.dt = &st->dt_corr;
  r.active = false;
  return ctx->launched(ctx->L->correct(a), "fused: correct");
}

adg_status adg_run_fused(adg_ctx* ctx, double* d_Q, const double* d_params, int32_t nsteps,
                         double cfl, double c_dt, int32_t creeping, double* d_dt_used,
                         int32_t* d_reruns, int32_t* d_flag) {
  if (!ctx) { g_err = "ctx is NULL"; return ADG_ERR_INVALID_ARG; }
  if (nsteps < 1) return ctx->fail(ADG_ERR_INVALID_ARG, "nsteps must be at least 1");
  adg_status s = adg_fused_begin(ctx, d_Q, d_params, cfl, c_dt, creeping, d_dt_used, nsteps,
                                 d_reruns, d_flag);
  for (int32_t k = 1; s == ADG_OK && k < nsteps; ++k) s = adg_fused_sweep(ctx);
  if (s != ADG_OK) {
    ctx->fz.active = false;
    return s;
  }
  return adg_fused_end(ctx);
}

static adg_status fv_check(adg_ctx* ctx, const void* in, const void* out) {
  if (!ctx) { g_err = "ctx is NULL"; return ADG_ERR_INVALID_ARG; }
  if (ctx->static_ws)
    return ctx->fail(ADG_ERR_WORKSPACE, "context has no workspace: only adg_step_noalloc runs on it");
  if (!in || !out) return ctx->fail(ADG_ERR_INVALID_ARG, "input and output buffers are required");
  if (!aligned16(in) || !aligned16(out))
    return ctx->fail(ADG_ERR_INVALID_ARG, "device buffers must be 16-byte aligned");
  if (in == out) return ctx->fail(ADG_ERR_INVALID_ARG, "input and output must be distinct buffers");
  if (!ctx->L->fv_step)
    return ctx->fail(ADG_ERR_UNSUPPORTED, "subcell patches need precision ADG_FP64 and "
                                          "time-integrated traces");
  return ADG_OK;
}

adg_status adg_fv_project(adg_ctx* ctx, const double* d_Q, double* d_P) {
  adg_status s = fv_check(ctx, d_Q, d_P);
  if (s != ADG_OK) return s;
  adg::LaunchArgs a = ctx->args();
  a.qin = d_Q;
  a.qout = d_P;
  return ctx->launched(ctx->L->fv_project(a), "fv_project");
}

adg_status adg_fv_reconstruct(adg_ctx* ctx, const double* d_P, double* d_Q) {
  adg_status s = fv_check(ctx, d_P, d_Q);
  if (s != ADG_OK) return s;
  adg::LaunchArgs a = ctx->args();
  a.qin = d_P;
  a.qout = d_Q;
  return ctx->launched(ctx->L->fv_reconstruct(a), "fv_reconstruct");
}

adg_status adg_fv_step(adg_ctx* ctx, const double* d_P, double* d_Pout, const double* d_params,
                       const double* d_dt, int32_t* d_flag) {
  adg_status s = fv_check(ctx, d_P, d_Pout);
  if (s != ADG_OK) return s;
  if (!d_dt) return ctx->fail(ADG_ERR_INVALID_ARG, "dt is required");
  if (n_params(ctx->cfg.pde) > 0 && !d_params)
    return ctx->fail(ADG_ERR_INVALID_ARG, "this PDE needs per-cell params");
  if (d_params && !aligned16(d_params))
    return ctx->fail(ADG_ERR_INVALID_ARG, "device buffers must be 16-byte aligned");
  adg::LaunchArgs a = ctx->args();
  a.qin = d_P;
  a.qout = d_Pout;
  a.params = d_params;
  a.dt = d_dt;
  a.flag = d_flag;
  return ctx->launched(ctx->L->fv_step(a), "fv_step");
}

adg_status adg_step_adjoint(adg_ctx* ctx, const double* d_Qn, const double* d_params, const double* d_dt,
                            double* d_Qbar, double* d_params_bar) {
  adg_status s = check_state(ctx, d_Qn, d_params, d_dt);
  if (s != ADG_OK) return s;
  if (!d_Qbar) return ctx->fail(ADG_ERR_INVALID_ARG, "Qbar is required");
  if (!ctx->L->adjoint) return ctx->fail(ADG_ERR_UNSUPPORTED, "adjoint needs precision ADG_FP64");
  if (ctx->lay.nslots <= 0)
    return ctx->fail(ADG_ERR_WORKSPACE, "adjoint workspace not reserved (set adg_config.adjoint)");
  adg::LaunchArgs a = ctx->args();
  a.Qc = d_Qn;
  a.params = d_params;
  a.dt = d_dt;
  a.Qbar = d_Qbar;
  a.params_bar = d_params_bar;
  return ctx->launched(ctx->L->adjoint(a), "adjoint");
}

}  // extern "C"
