"""GPU parity of the step with space-time traces and per-time-node Rusanov
(adg_config.spacetime_traces; Table 1's cardinalities) against the oracle."""

import pytest
import torch

from oracle import spacetime as ost
from oracle import step as ostep
from paper_1801_08682_amd import inputs
from paper_1801_08682_amd.inputs import ACOUSTIC, ADVECTION, ELASTIC, EULER
from tests.helpers import max_rel, setup_of

pytestmark = pytest.mark.gpu


def _wl(pde, d, N, nc, h=1.0 / 6.0, precision=inputs.FP64):
    pp = {EULER: (1.4,), ADVECTION: (1.0, -0.5, 0.3)[:d]}.get(pde, ())
    return inputs.Workload("st", pde, d, N, nc, nc[0] * h, pp, precision=precision)


CASES = [
    (EULER, 3, 3, (4, 3, 5), 0.2, 3),
    (EULER, 2, 4, (5, 6), 0.2, 3),
    (EULER, 3, 4, (3, 3, 4), 0.1, 2),
    (ACOUSTIC, 3, 2, (4, 3, 3), 1.0, 2),
    (ELASTIC, 2, 3, (5, 4), 1.0, 2),
    (ADVECTION, 2, 3, (5, 6), 1.0, 2),
    (EULER, 3, 7, (2, 2, 2), 0.1, 1),      # the gather-form predictor (n = 8)
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


@pytest.mark.parametrize("N,nc,prec", [
    (3, (4, 4, 3), inputs.FP64),
    (3, (4, 4, 3), inputs.FP32),
    (7, (2, 2, 2), inputs.FP64),
])
def test_spacetime_fused_matches_plain(N, nc, prec):
    """The fused sweep with space-time traces equals plain steps with the
    recorded dts (both on the GPU; the plain path is checked above): the
    same predictor, and the fused corrector's one-pass face solve takes the
    two-pass corrector's operands in the same order."""
    from paper_1801_08682_amd.stepper import Stepper
    wl = _wl(EULER, 3, N, nc, precision=prec)
    print(f"space-time fused vs plain N={N} grid={nc} precision={prec}", flush=True)
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


FLOAT_CASES = [
    (EULER, 3, 4, (4, 3, 3)),
    (EULER, 3, 7, (2, 2, 2)),
    (ELASTIC, 3, 5, (3, 2, 2)),
    (ACOUSTIC, 3, 3, (4, 3, 3)),
    (ADVECTION, 2, 3, (5, 6)),
]


@pytest.mark.parametrize("pde,d,N,nc", FLOAT_CASES)
def test_spacetime_float_predictor_matches_emulation(pde, d, N, nc):
    """The float predictor with space-time traces against the oracle's
    emulation (step_st_mixed "fp32"), element by element.  The float32
    quantities are those of the time-integrated float path, and each time
    node's traces are rounded once when stored, as the time-averaged ones
    are there, so the same derived bound holds: 8 u k max|Q| with u = 2^-24
    after k steps (the float predictor's parity test gives the derivation;
    the Rusanov flux of each time node enters with weight w_t, and the
    weights sum to one)."""
    from paper_1801_08682_amd.stepper import Stepper
    steps = 2
    wl = _wl(pde, d, N, nc, h=1.0 / 9.0, precision=inputs.FP32)
    Q0 = inputs.random_state(wl, seed=90 + N, amplitude=0.05)
    par = inputs.cell_params(wl, seed=91)
    s = setup_of(wl)
    Qt = torch.tensor(Q0)
    pt = None if par is None else torch.tensor(par)
    dt = ostep.cfl_dt(ostep.max_wave_speed(Qt, pt, s), 0.5 * inputs.stable_cfl(N), s)
    print(f"space-time float parity pde={pde} d={d} N={N} grid={nc} dt={dt}", flush=True)
    st = Stepper(wl, spacetime=True)
    Q = torch.tensor(Q0, device="cuda")
    p = None if par is None else torch.tensor(par, device="cuda")
    flag = torch.zeros(1, dtype=torch.int32, device="cuda")
    dtt = st.scalar(dt)
    for _ in range(steps):
        st.step(Q, p, dtt, flag)
    torch.cuda.synchronize()
    st.close()
    Qe = Qt
    for _ in range(steps):
        Qe = ost.step_st_mixed(Qe, pt, dt, s, "fp32")
    assert int(flag.item()) == 0
    dev = float((Q.cpu() - Qe).abs().max())
    scale = float(Qe.abs().max())
    print("max |gpu - emulation| / max|Q|", dev / scale, flush=True)
    assert dev <= 8 * 2.0 ** -24 * steps * scale

