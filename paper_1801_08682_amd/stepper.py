"""Python face of the C ABI: one context per stream over torch device buffers.

torch supplies device memory (``data_ptr()``) and the stream
(``torch.cuda.current_stream().cuda_stream``, a hipStream_t on ROCm); every
numerical step runs in libadg.so.  Names follow include/adg.h.
"""

import ctypes

import torch

from . import _lib
from .inputs import Workload


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


class Stepper:
    """ADER-DG stepper bound to one workload shape and one CUDA/HIP stream.

    Q: (ncells, (N+1)^d, m) float64 on the device, updated in place.
    params: (ncells, npar) float64 or None.  dt: float64 device tensor (1,).
    """

    def __init__(self, wl: Workload, device="cuda", stream=None, adjoint=False, fused=False,
                 spacetime=False):
        self.wl = wl
        self.L = _lib.load()
        self.device = torch.device(device)
        self.cfg = _lib.make_config(wl.dim, wl.order, wl.n_cells,
                                    [wl.length * wl.n_cells[i] / wl.n_cells[0]
                                     for i in range(wl.dim)],
                                    wl.pde, wl.pde_param, wl.picard_iters, wl.precision,
                                    adjoint, fused, spacetime)
        self.dofs_per_cell, self.npar, self.ws_bytes = _lib.query(self.cfg)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        with torch.cuda.stream(self.stream):
            self.workspace = torch.empty(max(self.ws_bytes, 256), dtype=torch.uint8,
                                         device=self.device)
        self.ctx = ctypes.c_void_p()
        _lib.check(self.L.adg_init(ctypes.byref(self.cfg), _ptr(self.workspace),
                                   self.ws_bytes, ctypes.c_void_p(self.stream.cuda_stream),
                                   ctypes.byref(self.ctx)))

    # -- argument checks (host side; the library validates again) --
    def _q(self, Q):
        wl = self.wl
        want = (wl.ncells, wl.n ** wl.dim, wl.m)
        if Q.dtype != torch.float64 or not Q.is_contiguous() or tuple(Q.shape) != want \
                or Q.device.type != "cuda":
            raise ValueError(f"Q must be a contiguous float64 device tensor of shape {want}")
        return _ptr(Q)

    def _p(self, params):
        if self.npar == 0:
            return None
        if params is None or params.dtype != torch.float64 or not params.is_contiguous() \
                or tuple(params.shape) != (self.wl.ncells, self.npar):
            raise ValueError(f"params must be float64 ({self.wl.ncells}, {self.npar})")
        return _ptr(params)

    def _check(self, st):
        _lib.check(st, self.ctx)

    # -- entry points --
    def predict(self, Q, params, dt):
        self._check(self.L.adg_predict(self.ctx, self._q(Q), self._p(params), _ptr(dt)))

    def correct(self, Q, params, dt, flag=None):
        self._check(self.L.adg_correct(self.ctx, self._q(Q), self._p(params), _ptr(dt),
                                       _ptr(flag)))

    def step(self, Q, params, dt, flag=None):
        self._check(self.L.adg_step(self.ctx, self._q(Q), self._p(params), _ptr(dt), _ptr(flag)))

    def wave_speed(self, Q, params):
        self._check(self.L.adg_wave_speed(self.ctx, self._q(Q), self._p(params)))

    def cfl_dt(self, cfl, lam=None, dt=None):
        self._check(self.L.adg_cfl_dt(self.ctx, float(cfl), _ptr(lam), _ptr(dt)))

    def step_adjoint(self, Qn, params, dt, Qbar, params_bar=None):
        self._q(Qbar)
        if params_bar is not None and self.npar:
            self._p(params_bar)
        self._check(self.L.adg_step_adjoint(self.ctx, self._q(Qn), self._p(params), _ptr(dt),
                                            _ptr(Qbar), _ptr(params_bar)))

    def run_fused(self, Q, params, steps, cfl, c_dt=0.99, creeping=True, flag=None):
        """Shifted, fused, optimistic stepping (Alg. 2) over `steps` steps.
        Returns (dt_used (steps,) float64, reruns (1,) int32) device tensors."""
        dt_used = torch.empty(steps, dtype=torch.float64, device=self.device)
        reruns = torch.zeros(1, dtype=torch.int32, device=self.device)
        self._check(self.L.adg_run_fused(self.ctx, self._q(Q), self._p(params), int(steps),
                                         float(cfl), float(c_dt), 1 if creeping else 0,
                                         _ptr(dt_used), _ptr(reruns), _ptr(flag)))
        return dt_used, reruns

    def fused_begin(self, Q, params, cfl, c_dt=0.99, creeping=True, capacity=0, flag=None):
        """adg_fused_begin; returns (dt_used (capacity,), reruns (1,)) device tensors."""
        dt_used = torch.empty(max(capacity, 1), dtype=torch.float64, device=self.device)
        reruns = torch.zeros(1, dtype=torch.int32, device=self.device)
        self._check(self.L.adg_fused_begin(self.ctx, self._q(Q), self._p(params), float(cfl),
                                           float(c_dt), 1 if creeping else 0,
                                           _ptr(dt_used) if capacity else None, int(capacity),
                                           _ptr(reruns), _ptr(flag)))
        return dt_used, reruns

    def fused_sweep(self):
        self._check(self.L.adg_fused_sweep(self.ctx))

    def fused_end(self):
        self._check(self.L.adg_fused_end(self.ctx))

    # -- finite-volume subcell patches (S = 2N + 1 subcells per axis) --
    @property
    def subcells(self):
        return 2 * self.wl.order + 1

    def _patch(self, P):
        wl = self.wl
        want = (wl.ncells, self.subcells ** wl.dim, wl.m)
        if P.dtype != torch.float64 or not P.is_contiguous() or tuple(P.shape) != want \
                or P.device.type != "cuda":
            raise ValueError(f"patches must be a contiguous float64 device tensor of shape {want}")
        return _ptr(P)

    def fv_project(self, Q, P):
        self._check(self.L.adg_fv_project(self.ctx, self._q(Q), self._patch(P)))

    def fv_reconstruct(self, P, Q):
        self._check(self.L.adg_fv_reconstruct(self.ctx, self._patch(P), self._q(Q)))

    def fv_step(self, P, Pout, params, dt, flag=None):
        self._check(self.L.adg_fv_step(self.ctx, self._patch(P), self._patch(Pout),
                                       self._p(params), _ptr(dt), _ptr(flag)))

    def close(self):
        if self.ctx:
            self.L.adg_destroy(self.ctx)
            self.ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- conveniences --
    def scalar(self, value=0.0):
        return torch.full((1,), float(value), dtype=torch.float64, device=self.device)

    def run(self, Q, params, steps, cfl=None, dt=None, flag=None, record_dt=False):
        """Alg. 1 (left): `steps` steps; dt fixed (a device scalar) or recomputed
        on the device from the state at the start of each step when `cfl` is
        given.  Returns the list of dt tensors when record_dt."""
        rec = []
        if cfl is not None:
            dtt = self.scalar()
            self.wave_speed(Q, params)
            self.cfl_dt(cfl, None, dtt)
        else:
            dtt = dt if torch.is_tensor(dt) else self.scalar(dt)
        for _ in range(steps):
            if record_dt:
                rec.append(dtt.clone())
            self.step(Q, params, dtt, flag)
            if cfl is not None:
                self.cfl_dt(cfl, None, dtt)
        return rec
