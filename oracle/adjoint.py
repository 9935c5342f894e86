"""Reverse mode through a rollout of oracle steps (torch autograd).

Oracle (test infrastructure only).  The time-step sequence is held fixed
(detached), as the hand-written GPU adjoint does.  Functionals:

* receiver misfit  J = 1/2 sum_n sum_r (p_h(x_r, t_n) - d_{r,n})^2, with
  p_h the DG polynomial of the first variable evaluated at the receiver
  (point values of the nodal basis, Sec. 3);
* final kinetic energy  KE(Q_N) = sum_c h^d sum_a W_a |j|^2 / (2 rho).

``grad_final_ke_mixed`` takes the forward steps with a reduced-precision
predictor (``mixed.step_mixed``) and differentiates with the float64 step's
linearisation at those states (the reverse sweep of the chain rule, one
``step_vjp`` per step from the last to the first).
"""

import torch

from . import mixed
from . import step as ostep
from .diagnostics import basis_rows, kinetic_energy


def rollout(Q0, par, s, dts, sample=None):
    """States after every step (list) and, if `sample` is given, the stacked
    samples sample(Q_n) for n = 1..len(dts)."""
    Q = Q0
    out = []
    for dt in dts:
        Q = ostep.step(Q, par, float(dt), s)
        if sample is not None:
            out.append(sample(Q))
    return Q, (torch.stack(out) if out else None)


def receiver_sampler(s, points, var=0):
    cells, rows = basis_rows(s, points)
    cells = torch.as_tensor(cells)

    def sample(Q):
        return (rows * Q[cells, :, var]).sum(-1)
    return sample


def misfit(Q0, par, s, dts, points, data):
    """J = 1/2 sum (samples - data)^2 over all steps and receivers."""
    _, smp = rollout(Q0, par, s, dts, receiver_sampler(s, points))
    return 0.5 * ((smp - data) ** 2).sum()


def grad_misfit(Q0, par, s, dts, points, data):
    """(J, dJ/dQ0, dJ/dpar) by autograd."""
    Q0 = Q0.clone().requires_grad_(True)
    p = None if par is None else par.clone().requires_grad_(True)
    J = misfit(Q0, p, s, dts, points, data)
    gs = torch.autograd.grad(J, [Q0] + ([p] if p is not None else []))
    return float(J.detach()), gs[0], (gs[1] if p is not None else None)


def grad_final_ke(Q0, s, dts):
    """(KE(Q_N), dKE/dQ0) by autograd (Euler)."""
    Q0 = Q0.clone().requires_grad_(True)
    QN, _ = rollout(Q0, None, s, dts)
    J = kinetic_energy(QN, s)
    (g,) = torch.autograd.grad(J, [Q0])
    return float(J.detach()), g


def step_vjp(Q, par, dt, s, G):
    """(dJ/dQ, dJ/dpar) for J = <G, step(Q)> (one step)."""
    Q = Q.clone().requires_grad_(True)
    p = None if par is None else par.clone().requires_grad_(True)
    out = ostep.step(Q, p, float(dt), s)
    gs = torch.autograd.grad((out * G).sum(), [Q] + ([p] if p is not None else []))
    return gs[0], (gs[1] if p is not None else None)


def grad_final_ke_mixed(Q0, s, dts, precision):
    """(KE(Q_N), G_0) for the rollout Q_n = S_p(Q_{n-1}; dt_n) whose steps
    take the predictor in ``precision`` ("fp64", "fp32", "bf16"), with
    G_N = dKE/dQ at Q_N and G_{n-1} = (dS/dQ at Q_{n-1})^T G_n, S the float64
    step (Euler, no materials)."""
    states = [Q0]
    for dt in dts:
        states.append(mixed.step_mixed(states[-1], None, float(dt), s, precision))
    QN = states[-1].clone().requires_grad_(True)
    J = kinetic_energy(QN, s)
    (G,) = torch.autograd.grad(J, [QN])
    for n in range(len(dts), 0, -1):
        G, _ = step_vjp(states[n - 1], None, dts[n - 1], s, G)
    return float(J.detach()), G
