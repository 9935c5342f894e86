"""adg_step_noalloc (include/adg.h): the step with the library's static
scratch instead of a caller workspace, for callers that cannot allocate.

Its output must equal adg_step's on the same inputs: the same kernels run on
the same data, so Q, the admissibility flag and the wave-speed maximum are
compared bit for bit.  Two calls in a row, the second on a smaller grid
(the scratch keeps the first call's contents), then a third with per-cell
materials.  The host-side refusals need no kernel launch.
"""

import ctypes

import pytest
import torch

from paper_1801_08682_amd import _lib, inputs
from paper_1801_08682_amd.stepper import Stepper

pytestmark = pytest.mark.gpu

STATIC_MAX = 32 << 20


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _static_ctx(st):
    """A context without workspace for the stepper's configuration."""
    L = _lib.load()
    ctx = ctypes.c_void_p()
    _lib.check(L.adg_init(ctypes.byref(st.cfg), None, 0,
                          ctypes.c_void_p(st.stream.cuda_stream), ctypes.byref(ctx)))
    return ctx


def _compare(wl, seed):
    print(f"noalloc vs adg_step: pde {wl.pde} d {wl.dim} N {wl.order} cells {wl.n_cells} "
          f"seed {seed}", flush=True)
    L = _lib.load()
    st = Stepper(wl)
    assert st.ws_bytes <= STATIC_MAX
    Q0 = torch.tensor(inputs.random_state(wl, seed=seed), device="cuda")
    par = inputs.cell_params(wl, seed)
    par = None if par is None else torch.tensor(par, device="cuda")
    dt = st.scalar(2.0e-3 * wl.h)
    # reference: adg_step on a caller workspace, then the wave-speed maximum
    Qa = Q0.clone()
    fa = torch.zeros(1, dtype=torch.int32, device="cuda")
    lam_a = st.scalar()
    st.step(Qa, par, dt, fa)
    st.cfl_dt(1.0, lam_a, None)
    # the same step through the static scratch
    ctx = _static_ctx(st)
    try:
        Qb = Q0.clone()
        fb = torch.zeros(1, dtype=torch.int32, device="cuda")
        lam_b = st.scalar(-1.0)
        _lib.check(L.adg_step_noalloc(ctx, _ptr(Qb), _ptr(par), _ptr(dt), _ptr(fb),
                                      _ptr(lam_b)), ctx)
        torch.cuda.synchronize()
        assert torch.equal(Qa, Qb)
        assert int(fa.item()) == int(fb.item()) == 0
        assert float(lam_a.item()) == float(lam_b.item()) > 0.0
        assert not torch.equal(Qb, Q0)
        # the other entry points refuse a context without workspace, and the
        # no-allocation step refuses a context with one (host checks only)
        st_ = L.adg_step(ctx, _ptr(Qb), _ptr(par), _ptr(dt), _ptr(fb))
        assert st_ == _lib.ADG_ERR_WORKSPACE
        st_ = L.adg_step_noalloc(st.ctx, _ptr(Qb), _ptr(par), _ptr(dt), _ptr(fb), None)
        assert st_ == _lib.ADG_ERR_WORKSPACE
    finally:
        L.adg_destroy(ctx)
        st.close()


def test_noalloc_matches_step_two_calls_second_smaller():
    big = inputs.Workload("na1", inputs.EULER, 3, 3, (6, 5, 4), 6 / 11, (1.4,))
    small = inputs.Workload("na2", inputs.EULER, 3, 3, (3, 3, 2), 3 / 11, (1.4,))
    _compare(big, 11)
    _compare(small, 12)


def test_noalloc_with_materials():
    wl = inputs.Workload("na3", inputs.ACOUSTIC, 3, 4, (4, 3, 5), 4 / 9)
    _compare(wl, 13)


def test_noalloc_refuses_grids_beyond_the_static_maximum():
    L = _lib.load()
    wl = inputs.preset("C2")                      # 6.4 GB of hull
    cfg = _lib.make_config(wl.dim, wl.order, wl.n_cells, [wl.length] * wl.dim, wl.pde,
                           wl.pde_param)
    ctx = ctypes.c_void_p()
    st = L.adg_init(ctypes.byref(cfg), None, 0, None, ctypes.byref(ctx))
    assert st == _lib.ADG_ERR_WORKSPACE
    assert "static maximum" in L.adg_last_error(None).decode()
    cfg = _lib.make_config(3, 3, (4, 4, 4), [1.0] * 3, inputs.EULER, (1.4,), fused=True)
    assert L.adg_init(ctypes.byref(cfg), None, 0, None, ctypes.byref(ctx)) == \
        _lib.ADG_ERR_INVALID_ARG
