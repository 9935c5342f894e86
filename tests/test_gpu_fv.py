"""GPU parity of the finite-volume subcell patches (include/adg.h:
adg_fv_project, adg_fv_reconstruct, adg_fv_step) against the oracle's
(oracle/fv.py), element-wise at the float64 bar (1e-12 relative), and
conservation of the totals on the device."""

import numpy as np
import pytest
import torch

from oracle import fv, step as ostep
from oracle.diagnostics import totals
from paper_1801_08682_amd import inputs
from paper_1801_08682_amd.inputs import ACOUSTIC, ADVECTION, ELASTIC, EULER
from tests.helpers import setup_of

pytestmark = pytest.mark.gpu
TOL64 = 1e-12


def _case(pde, d, N, nc, seed):
    pp = {EULER: (1.4,), ADVECTION: (1.0, -0.5, 0.25)[:d]}.get(pde, ())
    wl = inputs.Workload("fv", pde, d, N, tuple(nc), nc[0] / 5.0, pp)
    Q0 = inputs.random_state(wl, seed=seed, amplitude=0.05)
    par = inputs.cell_params(wl, seed=seed + 1)
    return wl, Q0, par


CASES = [(EULER, 3, 4, (3, 2, 2)), (EULER, 2, 3, (4, 3)), (EULER, 3, 1, (2, 3, 2)),
         (ACOUSTIC, 3, 3, (2, 2, 3)), (ELASTIC, 3, 2, (2, 2, 2)), (ADVECTION, 2, 0, (5, 3)),
         (EULER, 3, 7, (1, 2, 1))]


@pytest.mark.parametrize("pde,d,N,nc", CASES)
def test_patches_match_oracle(pde, d, N, nc):
    """Project the DG state onto the patches, take three subgrid steps (the
    dt of the subgrid from adg_cfl_dt after the first), reconstruct: every
    stage against the oracle."""
    from paper_1801_08682_amd.stepper import Stepper
    wl, Q0, par = _case(pde, d, N, nc, seed=90 + N)
    s = setup_of(wl)
    print("case fv patches", pde, d, N, nc, flush=True)
    st = Stepper(wl)
    S = st.subcells
    Q = torch.tensor(Q0, device="cuda")
    pd = None if par is None else torch.tensor(par, device="cuda")
    P = torch.empty(wl.ncells, S ** d, wl.m, dtype=torch.float64, device="cuda")
    P2 = torch.empty_like(P)
    st.fv_project(Q, P)
    Qt, pt = torch.tensor(Q0), None if par is None else torch.tensor(par)
    Pref = fv.project(Qt, s)
    assert float((P.cpu() - Pref).abs().max()) <= TOL64 * float(Pref.abs().max())
    flag = torch.zeros(1, dtype=torch.int32, device="cuda")
    dt = st.scalar(0.1 * s.h / S / d)
    dts = []
    for k in range(3):
        dts.append(float(dt.item()))
        st.fv_step(P, P2, pd, dt, flag)
        P, P2 = P2, P
        st.cfl_dt(0.5, None, dt)                     # the subgrid's admissible step
    torch.cuda.synchronize()
    for k in range(3):
        Pref = fv.fv_step(Pref, pt, dts[k], s)
        if k == 0:
            # after the first step: adg_cfl_dt gives 0.5 (h/S) / (d lambda_max)
            lam = max(float(s.pde.speed(fv.to_fine(Pref, s), i,
                                        None if pt is None else fv.to_fine(
                                            pt.reshape(pt.shape[0], 1, -1).expand(
                                                pt.shape[0], S ** d, pt.shape[-1]), s)).max())
                      for i in range(d))
            assert abs(dts[1] - 0.5 * (s.h / S) / (d * lam)) <= 1e-13 * dts[1]
    assert int(flag.item()) == 0
    err = float((P.cpu() - Pref).abs().max()) / float(Pref.abs().max())
    print("fv step max rel err", err)
    assert err <= TOL64
    # totals: sum of subcell averages times the subcell volume
    tot = lambda X: X.sum(dim=(0, 1)) * (s.h / S) ** d
    T0 = tot(fv.project(Qt, s))
    assert float((tot(P.cpu()) - T0).abs().max()) <= 1e-13 * (1.0 + float(T0.abs().max()))
    Qb = torch.empty_like(Q)
    st.fv_reconstruct(P, Qb)
    torch.cuda.synchronize()
    Qref = fv.reconstruct(Pref, s)
    assert float((Qb.cpu() - Qref).abs().max()) <= TOL64 * float(Qref.abs().max())
    st.close()


def test_patch_entry_points_refuse_bad_arguments():
    from paper_1801_08682_amd import _lib
    from paper_1801_08682_amd.stepper import Stepper
    wl, Q0, _ = _case(EULER, 3, 2, (2, 2, 2), seed=5)
    st = Stepper(wl)
    Q = torch.tensor(Q0, device="cuda")
    L = _lib.load()
    assert L.adg_fv_project(st.ctx, None, None) == _lib.ADG_ERR_INVALID_ARG
    p = Q.data_ptr()
    assert L.adg_fv_step(st.ctx, p, p, None, p, None) == _lib.ADG_ERR_INVALID_ARG   # in place
    st.close()
    st32 = Stepper(wl.with_(precision=inputs.FP32))
    P = torch.empty(wl.ncells, 125, wl.m, dtype=torch.float64, device="cuda")
    assert L.adg_fv_project(st32.ctx, Q.data_ptr(), P.data_ptr()) == _lib.ADG_ERR_UNSUPPORTED
    st32.close()
