"""Differentiable rollout over the C ABI (adg_step forward, adg_step_adjoint
backward) with checkpoint-every-k recomputation.

Forward: Q_n = S(Q_{n-1}; dt_n) for n = 1..N on the device; dt_n fixed or
recomputed on the device from Q_{n-1} (calcTimeStep, Sec. 3) and recorded.
States are kept every k steps.  Optional receivers sample the DG polynomial
of variable 0 at fixed points after every step (point values of the nodal
basis: row . Q[cell]); the rows are host-built and passed in.

Backward: for each checkpoint segment in reverse, recompute its states with
adg_step, then apply adg_step_adjoint from the last step of the segment to the
first, adding the receiver seeds.  The recorded dt sequence is held fixed.

Reduced-precision forward: with a second stepper of the same grid whose
predictor runs in float or bfloat16 (``forward=``), that stepper takes the
forward steps and the segment recomputes, and the float64 adjoint steps are
applied at its states: the gradient is the float64 linearisation of the step
along the reduced-precision trajectory.
"""

import torch

from .stepper import Stepper


class _Rollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, Q0, params, st, fw, nsteps, dt, cfl, k, rec_cells, rec_rows):
        par = params if params.numel() else None
        Q = Q0.detach().clone()
        dts, ckpt = [], {0: Q0.detach().clone()}
        dtt = fw.scalar() if cfl is not None else (dt if torch.is_tensor(dt) else fw.scalar(dt))
        if cfl is not None:
            fw.wave_speed(Q, par)
            fw.cfl_dt(cfl, None, dtt)
        samples = []
        for n in range(1, nsteps + 1):
            dts.append(dtt.clone())
            fw.step(Q, par, dtt)
            if cfl is not None:
                fw.cfl_dt(cfl, None, dtt)
            if rec_cells is not None:
                samples.append((rec_rows * Q[rec_cells, :, 0]).sum(-1))
            if n % k == 0 and n < nsteps:
                ckpt[n] = Q.clone()
        ctx.st, ctx.fw, ctx.dts, ctx.ckpt, ctx.k, ctx.nsteps = st, fw, dts, ckpt, k, nsteps
        ctx.par = par
        ctx.rec = (rec_cells, rec_rows)
        S = torch.stack(samples) if samples else torch.zeros(0, device=Q.device, dtype=Q.dtype)
        return Q, S

    @staticmethod
    def backward(ctx, gQ, gS):
        st, fw, dts, k, N, par = ctx.st, ctx.fw, ctx.dts, ctx.k, ctx.nsteps, ctx.par
        rec_cells, rec_rows = ctx.rec
        Qbar = torch.zeros_like(ctx.ckpt[0]) if gQ is None else gQ.contiguous().clone()
        pbar = None if par is None else torch.zeros_like(par)

        def seed(n):      # receiver seed of the sample of Q_n (n >= 1)
            if rec_cells is not None and gS is not None and gS.numel():
                Qbar[:, :, 0].index_put_((rec_cells,), rec_rows * gS[n - 1][:, None],
                                         accumulate=True)

        seed(N)
        starts = sorted(ctx.ckpt.keys())
        for s0 in reversed(starts):
            s1 = min(s0 + k, N)
            states = [ctx.ckpt[s0].clone()]
            for n in range(s0 + 1, s1):
                Q = states[-1].clone()
                fw.step(Q, par, dts[n - 1])
                states.append(Q)
            for n in range(s1, s0, -1):
                st.step_adjoint(states[n - 1 - s0], par, dts[n - 1], Qbar, pbar)
                if n - 1 >= 1:
                    seed(n - 1)
        return (Qbar, pbar if pbar is not None else None, None, None, None, None, None, None, None,
                None)


def rollout(st: Stepper, Q0, params, nsteps, dt=None, cfl=None, checkpoint_every=10,
            receivers=None, forward=None):
    """Differentiable N-step rollout.

    st: a Stepper created with adjoint=True (float64).  Q0 (and params) may
    require grad.  receivers: None or (cells LongTensor (R,), rows (R, nn))
    on the device.  forward: None (st steps forward too) or a Stepper of the
    same grid and PDE with a reduced-precision predictor, which takes the
    forward steps and the recomputes.  Returns (Q_N, samples (N, R) or empty).
    """
    if (dt is None) == (cfl is None):
        raise ValueError("give exactly one of dt and cfl")
    fw = st if forward is None else forward
    if fw is not st:
        a, b = fw.wl, st.wl
        if (a.pde, a.dim, a.order, tuple(a.n_cells), a.length, tuple(a.pde_param), a.picard_iters) != \
                (b.pde, b.dim, b.order, tuple(b.n_cells), b.length, tuple(b.pde_param), b.picard_iters):
            raise ValueError("the forward stepper must have the adjoint stepper's grid and PDE")
    params_t = params if params is not None else torch.zeros(0, dtype=Q0.dtype, device=Q0.device)
    rc, rr = receivers if receivers is not None else (None, None)
    return _Rollout.apply(Q0, params_t, st, fw, nsteps, dt, cfl, int(checkpoint_every), rc, rr)


def kinetic_energy(Q, dim, h, w1d):
    """KE = sum_c h^d sum_a W_a |j|^2 / (2 rho) on the device (Euler);
    w1d: the 1D Gauss-Legendre weights on [0, 1] as a device tensor."""
    W = w1d
    for _ in range(dim - 1):
        W = torch.kron(w1d, W)
    j = Q[..., 1:1 + dim]
    return (h ** dim) * (W * 0.5 * (j * j).sum(-1) / Q[..., 0]).sum()


def receiver_rows(wl, points):
    """Cells and nodal-basis rows that sample the DG polynomial at physical
    points: value = rows[r] . Q[cells[r], :, var].  Lagrange basis on the
    Gauss-Legendre nodes by the product formula."""
    import numpy as np
    n, d, h = wl.n, wl.dim, wl.h
    z, _ = np.polynomial.legendre.leggauss(n)
    xi = 0.5 * (1.0 + z)
    cells, rows = [], []
    for x in np.asarray(points, dtype=np.float64):
        idx, row = [], np.ones(1)
        for i in range(d):
            L = wl.n_cells[i] * h
            s = (x[i] % L) / h
            ci = min(int(np.floor(s)), wl.n_cells[i] - 1)
            t = s - ci
            phi = np.array([np.prod([(t - xi[k]) / (xi[j] - xi[k]) for k in range(n) if k != j])
                            for j in range(n)])
            idx.append(ci)
            row = np.kron(phi, row)
        c = 0
        for i in reversed(range(d)):
            c = c * wl.n_cells[i] + idx[i]
        cells.append(c)
        rows.append(row)
    return np.array(cells, dtype=np.int64), np.array(rows)
