"""GPU parity of the step with space-time traces and per-time-node Rusanov
(adg_config.spacetime_traces; Table 1's cardinalities) against the oracle."""

import pytest
import torch

from oracle import spacetime as ost
from paper_1801_08682_amd import inputs
from paper_1801_08682_amd.inputs import ACOUSTIC, ADVECTION, ELASTIC, EULER
from tests.helpers import max_rel, setup_of

pytestmark = pytest.mark.gpu


def _wl(pde, d, N, nc):
    h = 1.0 / 6.0
    pp = {EULER: (1.4,), ADVECTION: (1.0, -0.5, 0.3)[:d]}.get(pde, ())
    return inputs.Workload("st", pde, d, N, nc, nc[0] * h, pp)


CASES = [
    (EULER, 3, 3, (4, 3, 5), 0.2, 3),
    (EULER, 2, 4, (5, 6), 0.2, 3),
    (EULER, 3, 4, (3, 3, 4), 0.1, 2),
    (ACOUSTIC, 3, 2, (4, 3, 3), 1.0, 2),
    (ELASTIC, 2, 3, (5, 4), 1.0, 2),
    (ADVECTION, 2, 3, (5, 6), 1.0, 2),
]


@pytest.mark.parametrize("pde,d,N,nc,amp,steps", CASES)
def test_spacetime_matches_oracle(pde, d, N, nc, amp, steps):
    from paper_1801_08682_amd.stepper import Stepper
    wl = _wl(pde, d, N, nc)
    Q0 = inputs.random_state(wl, seed=8, amplitude=amp)
    par = inputs.cell_params(wl, seed=8)
    dt = 0.2 * wl.h / (d * (2 * N + 1))
    print(f"space-time parity pde={pde} d={d} N={N} grid={nc}", flush=True)
    st = Stepper(wl, spacetime=True)
    Q = torch.tensor(Q0, device="cuda")
    p = None if par is None else torch.tensor(par, device="cuda")
    flag = torch.zeros(1, dtype=torch.int32, device="cuda")
    dtt = st.scalar(dt)
    for _ in range(steps):
        st.step(Q, p, dtt, flag)
    torch.cuda.synchronize()
    st.close()
    s = setup_of(wl)
    QO = torch.tensor(Q0)
    pO = None if par is None else torch.tensor(par)
    for _ in range(steps):
        QO = ost.step_st(QO, pO, dt, s)
    assert int(flag.item()) == 0
    assert max_rel(Q.cpu(), QO, wl) < 1e-12


def test_spacetime_fused_matches_plain():
    """The fused sweep with space-time traces equals plain steps with the
    recorded dts (both on the GPU; the plain path is checked above)."""
    from paper_1801_08682_amd.stepper import Stepper
    wl = _wl(EULER, 3, 3, (4, 4, 3))
    Q0 = torch.tensor(inputs.random_state(wl, seed=9, amplitude=0.2), device="cuda")
    st = Stepper(wl, fused=True, spacetime=True)
    Q = Q0.clone()
    used, reruns = st.run_fused(Q, None, 4, 0.5, 0.99)
    QP = Q0.clone()
    for dt in used.cpu().tolist():
        st.step(QP, None, st.scalar(dt))
    torch.cuda.synchronize()
    st.close()
    assert float((Q - QP).abs().max()) < 1e-13 * float(QP.abs().max())


def test_spacetime_has_no_adjoint():
    from paper_1801_08682_amd import _lib
    from paper_1801_08682_amd.stepper import Stepper
    wl = _wl(EULER, 2, 2, (3, 3))
    st = Stepper(wl, adjoint=True, spacetime=True)
    Q = torch.tensor(inputs.random_state(wl, seed=1), device="cuda")
    with pytest.raises(_lib.AdgError) as e:
        st.step_adjoint(Q, None, st.scalar(1e-3), Q.clone())
    assert e.value.status == _lib.ADG_ERR_UNSUPPORTED
    st.close()
