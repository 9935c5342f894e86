"""Oracle pins of the step with space-time traces and a Rusanov solve per
time node (Table 1's extrapolate / solveRiemann cardinalities), CPU only.

* Linear advection has a constant wave speed, so the Rusanov flux is linear
  in the traces and its time integral is that of the time-integrated traces:
  the space-time step equals the plain step.
* Conservation of the cell totals.
* A brute-force evaluation with explicit loops over cells, faces, time nodes
  and face nodes on a tiny Euler grid (the predictor and the volume term are
  taken from the oracle; they are pinned elsewhere).
* The reduced-precision form (step_st_mixed): unrounded it is the float64
  space-time step; in float32 a constant state stays constant, the totals
  are conserved and the error against float64 sits at the float32 scale.
"""

import numpy as np
import pytest
import torch

from oracle import spacetime as ost
from oracle import step as ostep
from oracle.diagnostics import l2, totals
from paper_1801_08682_amd import inputs
from paper_1801_08682_amd.inputs import ADVECTION, ACOUSTIC, ELASTIC, EULER


def _case(pde, d, N, nc, seed, amp):
    h = 1.0 / nc[0]
    pp = {EULER: (1.4,), ADVECTION: (1.0, -0.5, 0.3)[:d]}.get(pde, ())
    wl = inputs.Workload("st", pde, d, N, nc, nc[0] * h, pp)
    Q = torch.tensor(inputs.random_state(wl, seed=seed, amplitude=amp))
    par = inputs.cell_params(wl, seed=seed)
    return ostep.Setup(pde, d, N, nc, h, pp), Q, (None if par is None else torch.tensor(par))


@pytest.mark.parametrize("d,N,nc", [(2, 3, (4, 3)), (3, 2, (3, 2, 3))])
def test_advection_equals_time_integrated_step(d, N, nc):
    s, Q, _ = _case(ADVECTION, d, N, nc, seed=1, amp=1.0)
    dt = 0.02
    assert float((ost.step_st(Q, None, dt, s) - ostep.step(Q, None, dt, s)).abs().max()) < 1e-14


@pytest.mark.parametrize("pde,d,N,nc", [(EULER, 2, 3, (4, 3)), (ACOUSTIC, 3, 2, (3, 3, 2))])
def test_conservation(pde, d, N, nc):
    s, Q, par = _case(pde, d, N, nc, seed=2, amp=0.2 if pde == EULER else 1.0)
    Qn = ost.step_st(Q, par, 0.01, s)
    assert torch.allclose(totals(Qn, s), totals(Q, s), rtol=0, atol=1e-13)


def test_euler_brute_force():
    s, Q, _ = _case(EULER, 2, 2, (3, 2), seed=3, amp=0.3)
    n, m, h, dt = s.n, s.m, s.h, 0.03
    C = Q.shape[0]
    u = ostep._spatial(Q, s)
    q = ostep.predictor(u, None, dt, s)                       # (C, t, k1, k0, m)
    _, Fbar = ostep.time_average(q, None, s)
    Qt = ostep.integrate_volume(u, Fbar, dt, s).numpy()      # (C, k1, k0, m)
    qn = q.numpy()
    FL, FR, w, LL, LR = (np.asarray(x) for x in (s.tab.FL, s.tab.FR, s.tab.w, s.tab.LL, s.tab.LR))
    plus, _ = ostep.neighbor_index(s.n_cells)

    def node(c, t, i, b, j):          # q at time t, coordinate j along axis i, face node b
        return qn[c, t, b, j] if i == 0 else qn[c, t, j, b]

    def flux(v, i):
        return s.pde.flux(torch.tensor(v), i, None).numpy()

    def speed(v, i):
        return float(s.pde.speed(torch.tensor(v), i, None))

    Fstar = np.zeros((2, C, n, m))    # [axis][left cell][face node][var]: F* on its + face
    for i in range(2):
        for c in range(C):
            cp = plus[i][c]
            Ft = np.zeros((n, n, m))
            for t in range(n):
                qL = [sum(FR[j] * node(c, t, i, b, j) for j in range(n)) for b in range(n)]
                qR = [sum(FL[j] * node(cp, t, i, b, j) for j in range(n)) for b in range(n)]
                fL = [sum(FR[j] * flux(node(c, t, i, b, j), i) for j in range(n)) for b in range(n)]
                fR = [sum(FL[j] * flux(node(cp, t, i, b, j), i) for j in range(n)) for b in range(n)]
                sm = max(max(speed(qL[b], i), speed(qR[b], i)) for b in range(n))
                for b in range(n):
                    Ft[t, b] = 0.5 * (fL[b] + fR[b]) - 0.5 * sm * (qR[b] - qL[b])
            Fstar[i, c] = sum(w[t] * Ft[t] for t in range(n))
    minus = [np.argsort(plus[i]) for i in range(2)]
    ref = Qt.copy()
    for c in range(C):
        for k1 in range(n):
            for k0 in range(n):
                ref[c, k1, k0] -= dt / h * (LR[k0] * Fstar[0, c, k1] - LL[k0] * Fstar[0, minus[0][c], k1])
                ref[c, k1, k0] -= dt / h * (LR[k1] * Fstar[1, c, k0] - LL[k1] * Fstar[1, minus[1][c], k0])
    got = ost.step_st(Q, None, dt, s).numpy().reshape(C, n, n, m)
    assert np.abs(got - ref).max() < 1e-13
    # and the per-time-node solve differs from the time-integrated one
    assert np.abs(got - ostep.step(Q, None, dt, s).numpy().reshape(C, n, n, m)).max() > 1e-9


# The reduced-precision space-time step: pinned like the plain mixed step
# (its unrounded arrangement is the float64 space-time step above; a constant
# state stays constant and the totals are conserved in any precision; the
# float32 error sits at the float32 scale).
MIXED_CASES = [(EULER, 2, 3, (4, 3)), (ACOUSTIC, 3, 2, (3, 3, 2)), (ELASTIC, 2, 2, (3, 4))]


def _mixed_case(pde, d, N, nc):
    s, Q, par = _case(pde, d, N, nc, seed=5, amp=0.05 if pde == EULER else 1.0)
    dt = ostep.cfl_dt(ostep.max_wave_speed(Q, par, s), 0.5 * inputs.stable_cfl(N), s)
    return s, Q, par, dt


@pytest.mark.parametrize("pde,d,N,nc", MIXED_CASES)
def test_mixed_unrounded_arrangement_is_the_plain_st_step(pde, d, N, nc):
    s, Q, par, dt = _mixed_case(pde, d, N, nc)
    a = ost.step_st_mixed(Q, par, dt, s, "fp64")
    b = ost.step_st(Q, par, dt, s)
    assert float((l2(a - b, s) / l2(b - Q, s)).max()) < 1e-12


@pytest.mark.parametrize("pde,d,N,nc", MIXED_CASES)
def test_mixed_st_invariants_and_error_size(pde, d, N, nc):
    s, Q, par, dt = _mixed_case(pde, d, N, nc)
    c = Q[0:1, 0:1].expand_as(Q).clone()
    pc = None if par is None else par[0:1].expand_as(par).clone()
    out = ost.step_st_mixed(c, pc, dt, s, "fp32")
    assert (out - c).abs().max() < 1e-13 * (1 + c.abs().max())
    M0 = totals(Q, s)
    out = ost.step_st_mixed(Q, par, dt, s, "fp32")
    assert (totals(out, s) - M0).abs().max() < 1e-14 * (1 + M0.abs().max())
    ref = ost.step_st(Q, par, dt, s)
    e32 = float((l2(out - ref, s) / l2(ref - Q, s)).max())
    assert 1e-9 < e32 < 256 * 2.0 ** -24
