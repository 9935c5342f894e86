"""GPU parity of the shifted, fused, optimistic stepping (adg_run_fused;
Sec. 5, Techniques 3-5; Alg. 2) against the oracle's Alg. 2, and against
plain adg_step with the same time steps."""

import numpy as np
import pytest
import torch

from oracle import fused as ofused
from paper_1801_08682_amd import inputs
from paper_1801_08682_amd.inputs import ACOUSTIC, ADVECTION, ELASTIC, EULER

from tests.helpers import max_rel, setup_of

pytestmark = pytest.mark.gpu


def _wl(pde, d, N, nc, prec=inputs.FP64):
    h = 1.0 / 6.0
    pp = {EULER: (1.4,), ADVECTION: (1.0, -0.5, 0.3)[:d]}.get(pde, ())
    return inputs.Workload("f", pde, d, N, nc, nc[0] * h, pp, precision=prec)


def _gpu_fused(wl, Q0, par, K, cfl, c_dt, creeping=True):
    from paper_1801_08682_amd.stepper import Stepper
    st = Stepper(wl, fused=True)
    Q = torch.tensor(Q0, device="cuda")
    p = None if par is None else torch.tensor(par, device="cuda")
    flag = torch.zeros(1, dtype=torch.int32, device="cuda")
    used, reruns = st.run_fused(Q, p, K, cfl, c_dt, creeping, flag)
    torch.cuda.synchronize()
    out = (Q.cpu(), used.cpu().numpy(), int(reruns.item()), int(flag.item()))
    st.close()
    return out


CASES = [
    # pde, d, N, grid, K, cfl, c_dt, creeping, amplitude
    (EULER, 3, 3, (4, 3, 5), 5, 0.6, 0.99, True, 0.2),
    (EULER, 2, 4, (6, 5), 5, 0.3, 1.5, True, 0.1),       # a rerun after every sweep
    (EULER, 3, 4, (3, 4, 3), 3, 0.5, 0.99, False, 0.2),
    (ACOUSTIC, 3, 2, (4, 3, 3), 4, 0.8, 0.99, True, 1.0),
    (ELASTIC, 2, 3, (5, 4), 4, 0.7, 0.99, True, 1.0),
    (ADVECTION, 2, 3, (5, 6), 4, 0.9, 0.99, True, 1.0),
    # one cell along an axis: the periodic neighbour is the cell itself
    (EULER, 3, 4, (1, 1, 1), 3, 0.5, 0.99, True, 0.2),
    (EULER, 3, 2, (1, 3, 2), 3, 0.5, 0.99, True, 0.2),
]


@pytest.mark.parametrize("pde,d,N,nc,K,cfl,c_dt,creeping,amp", CASES)
def test_fused_matches_oracle(pde, d, N, nc, K, cfl, c_dt, creeping, amp):
    wl = _wl(pde, d, N, nc)
    Q0 = inputs.random_state(wl, seed=5, amplitude=amp)
    par = inputs.cell_params(wl, seed=5)
    print(f"fused parity pde={pde} d={d} N={N} grid={nc} K={K} c_dt={c_dt}", flush=True)
    Q, used, reruns, flag = _gpu_fused(wl, Q0, par, K, cfl, c_dt, creeping)
    QO, usedO, rerunsO = ofused.run_fused(torch.tensor(Q0), None if par is None else torch.tensor(par),
                                          setup_of(wl), K, cfl, c_dt, creeping)
    assert flag == 0
    assert reruns == rerunsO
    if c_dt > 1:
        assert reruns == K - 1
    assert np.allclose(used, usedO, rtol=1e-12, atol=0)
    assert max_rel(Q, QO, wl) < 1e-12


def _plain(wl, Q0, par, dts):
    from paper_1801_08682_amd.stepper import Stepper
    st = Stepper(wl)
    Q = torch.tensor(Q0, device="cuda") if not torch.is_tensor(Q0) else Q0.clone()
    p = None if par is None else torch.as_tensor(par, device="cuda")
    for dt in dts:
        st.step(Q, p, st.scalar(float(dt)))
    torch.cuda.synchronize()
    st.close()
    return Q


def test_fused_float_predictor_tracks_plain_float_path():
    wl = _wl(EULER, 3, 4, (4, 5, 3), prec=inputs.FP32)
    Q0 = inputs.random_state(wl, seed=6, amplitude=0.2)
    Q, used, reruns, flag = _gpu_fused(wl, Q0, None, 4, 0.5, 0.99)
    QP = _plain(wl, Q0, None, used).cpu()
    assert flag == 0
    # both are float predictors whose kernels order (and contract to FMA)
    # their float arithmetic differently: per step they may differ by the
    # float rounding bound of the update, 8 u max|Q| with u = 2^-24 (the
    # derivation is in tests/test_gpu_precision.py)
    assert float((Q - QP).abs().max()) < 4 * 8 * 2.0 ** -24 * float(QP.abs().max())


@pytest.mark.parametrize("ic,steps", [("bump", 3), ("fourier", 10)])
def test_fused_full_size_c2_matches_plain_steps(ic, steps):
    """The benchmark's workload and launch configuration (81^3 cells, N = 4):
    fused steps equal plain steps with the same dts, on the bump (a
    stationary contact) and on a moving flow (Fourier density modes with
    p = rho^gamma, every field changing)."""
    wl = inputs.preset("C2").with_(extra={"ic": ic})
    Q0 = torch.tensor(inputs.initial_state(wl), device="cuda")
    print("fused C2 full size", ic, steps, flush=True)
    from paper_1801_08682_amd.stepper import Stepper
    st = Stepper(wl, fused=True)
    Q = Q0.clone()
    used, reruns = st.run_fused(Q, None, steps, wl.cfl, 0.99)
    torch.cuda.synchronize()
    st.close()
    QP = _plain(wl, Q0, None, used.cpu().numpy())
    err = float((Q - QP).abs().max()) / float(QP.abs().max())
    assert err < 1e-13
    assert int(reruns.item()) == 0


def test_run_fused_argument_errors():
    from paper_1801_08682_amd import _lib
    from paper_1801_08682_amd.stepper import Stepper
    wl = _wl(EULER, 2, 2, (3, 3))
    Q = torch.tensor(inputs.random_state(wl, seed=1), device="cuda")
    st = Stepper(wl)                       # no fused workspace
    with pytest.raises(_lib.AdgError) as e:
        st.run_fused(Q, None, 2, 0.5)
    assert e.value.status == _lib.ADG_ERR_WORKSPACE
    st.close()
    st = Stepper(wl, fused=True)
    with pytest.raises(_lib.AdgError) as e:
        st.run_fused(Q, None, 0, 0.5)
    assert e.value.status == _lib.ADG_ERR_INVALID_ARG
    st.close()


def test_begin_sweep_end_equals_run_fused():
    from paper_1801_08682_amd.stepper import Stepper
    wl = _wl(EULER, 3, 2, (4, 4, 3))
    Q0 = torch.tensor(inputs.random_state(wl, seed=7, amplitude=0.2), device="cuda")
    st = Stepper(wl, fused=True)
    A = Q0.clone()
    usedA, _ = st.run_fused(A, None, 4, 0.6)
    B = Q0.clone()
    usedB, rerB = st.fused_begin(B, None, 0.6, capacity=4)
    for _ in range(3):
        st.fused_sweep()
    st.fused_end()
    torch.cuda.synchronize()
    assert torch.equal(A, B)
    assert torch.equal(usedA, usedB)
    from paper_1801_08682_amd import _lib
    with pytest.raises(_lib.AdgError):
        st.fused_sweep()                      # the run has ended
    st.close()
