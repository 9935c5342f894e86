"""Oracle pins of the shifted, fused, optimistic stepping (Sec. 5,
Techniques 3-5; Alg. 2), CPU only.

The arithmetic of a step is pinned elsewhere; these tests pin the split of a
step at the hull and the time step control against what Alg. 2 states:
* the STP task followed by the corrector is the plain step;
* with a constant wave speed no rerun happens and the fused run is plain
  stepping with C_dT * Delta T_adm;
* every used step obeys the rule of Alg. 2: the creeping average of the
  previous step and C_dT Delta T_adm of the state before it, unless the new
  state does not admit it, in which case C_dT Delta T_adm of the new state;
* with C_dT <= 1 no used step exceeds the admissible step of the state it
  starts from (the CFL condition is never harmed);
* C_dT > 1 forces a rerun after every sweep.
"""

import numpy as np
import pytest
import torch

from oracle import fused as ofused
from oracle import step as ostep
from paper_1801_08682_amd import inputs
from paper_1801_08682_amd.inputs import ADVECTION, EULER


def _case(pde, d, N, nc, seed=0, amp=0.05):
    h = 1.0 / nc[0]
    pp = {EULER: (1.4,), ADVECTION: (1.0, -0.5, 0.3)[:d]}[pde]
    wl = inputs.Workload("f", pde, d, N, nc, nc[0] * h, pp)
    Q = torch.tensor(inputs.random_state(wl, seed=seed, amplitude=amp))
    return ostep.Setup(pde, d, N, nc, h, pp), Q


def _replay(Q, s, dts):
    """States Q^0..Q^K of plain steps with the given dts."""
    out = [Q]
    for dt in dts:
        out.append(ostep.step(out[-1], None, dt, s))
    return out


def test_stp_then_corrector_is_the_step():
    s, Q = _case(EULER, 2, 3, (4, 3), seed=1)
    dt = 0.3 * ofused.admissible_dt(Q, None, 0.5, s)
    Qt, tr = ofused.stp(Q, None, dt, s)
    Qn = ofused.corrector(Qt, tr, None, dt, s)
    assert torch.equal(Qn, ostep.step(Q, None, dt, s))


def test_constant_speed_no_rerun():
    s, Q = _case(ADVECTION, 2, 2, (4, 4), seed=2)
    cfl, c_dt = 0.9, 0.99
    QF, used, reruns = ofused.run_fused(Q, None, s, 4, cfl, c_dt)
    dt = c_dt * ofused.admissible_dt(Q, None, cfl, s)
    assert reruns == 0
    assert np.allclose(used, dt, rtol=1e-15, atol=0)
    QP, _ = ostep.run(Q, None, s, 4, dt=dt)
    assert float((QF - QP).abs().max()) < 1e-14


@pytest.mark.parametrize("c_dt,creeping", [(0.99, True), (0.99, False), (0.9, True)])
def test_used_steps_follow_alg2(c_dt, creeping):
    s, Q = _case(EULER, 2, 2, (4, 4), seed=3, amp=0.2)
    cfl, K = 0.6, 6
    _, used, reruns = ofused.run_fused(Q, None, s, K, cfl, c_dt, creeping)
    states = _replay(Q, s, used)
    adm = [ofused.admissible_dt(x, None, cfl, s) for x in states]
    assert used[0] == pytest.approx(c_dt * adm[0], rel=1e-15)
    nre = 0
    for k in range(1, K):
        planned = (0.5 * (used[k - 1] + c_dt * adm[k - 1]) if creeping else c_dt * adm[k - 1]) \
            if k > 1 else c_dt * adm[0]
        if adm[k] < planned:
            nre += 1
            assert used[k] == pytest.approx(c_dt * adm[k], rel=1e-14)
        else:
            assert used[k] == pytest.approx(planned, rel=1e-14)
        assert used[k] <= adm[k] * (1 + 1e-14)          # CFL never harmed
    assert nre == reruns


def test_forced_rerun_every_sweep():
    s, Q = _case(EULER, 2, 2, (3, 3), seed=4, amp=0.1)
    cfl, c_dt, K = 0.4, 1.5, 4
    _, used, reruns = ofused.run_fused(Q, None, s, K, cfl, c_dt)
    assert reruns == K - 1
    states = _replay(Q, s, used)
    for k in range(K):
        assert used[k] == pytest.approx(c_dt * ofused.admissible_dt(states[k], None, cfl, s),
                                        rel=1e-14)
