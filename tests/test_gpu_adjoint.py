"""GPU reverse mode: adg_step_adjoint against the oracle's autograd and
central finite differences; the checkpointed rollout (receiver misfit,
final kinetic energy) against the oracle's autograd through its rollout."""

import numpy as np
import pytest
import torch

from paper_1801_08682_amd import inputs
from paper_1801_08682_amd.rollout import rollout, receiver_rows, kinetic_energy
from paper_1801_08682_amd.stepper import Stepper
from oracle import adjoint as oadj
from oracle import step as ostep
from tests.helpers import setup_of

pytestmark = pytest.mark.gpu


def _wl(pde, dim, order, n_cells, pp=()):
    h = 1.0 / 8.0
    return inputs.Workload("adj", pde, dim, order, tuple(n_cells), n_cells[0] * h, tuple(pp))


CASES = [(inputs.EULER, 3, 2, (3, 2, 2), (1.4,)), (inputs.EULER, 2, 4, (3, 3), (1.4,)),
         (inputs.EULER, 3, 7, (2, 1, 1), (1.4,)), (inputs.ACOUSTIC, 3, 3, (3, 2, 2), ()),
         (inputs.ELASTIC, 3, 2, (2, 2, 2), ()), (inputs.ELASTIC, 2, 3, (3, 2), ()),
         (inputs.ADVECTION, 2, 3, (3, 3), (1.0, -0.5))]


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"pde{c[0]}d{c[1]}N{c[2]}")
def test_step_vjp_matches_oracle_autograd(case):
    pde, d, N, nc, pp = case
    wl = _wl(pde, d, N, nc, pp)
    rng = np.random.default_rng(5)
    Q = inputs.random_state(wl, seed=80 + N, amplitude=0.05)
    par = inputs.cell_params(wl, seed=1)
    G = rng.standard_normal(Q.shape)
    dt = 2e-3
    print("case vjp", case, flush=True)
    st = Stepper(wl, adjoint=True)
    Qd = torch.tensor(Q, device="cuda")
    pd = None if par is None else torch.tensor(par, device="cuda")
    Gd = torch.tensor(G, device="cuda")
    pbar = None if par is None else torch.zeros_like(pd)
    st.step_adjoint(Qd, pd, st.scalar(dt), Gd, pbar)
    torch.cuda.synchronize()
    assert torch.equal(Qd.cpu(), torch.tensor(Q))          # Q(T) untouched
    gq, gp = oadj.step_vjp(torch.tensor(Q), None if par is None else torch.tensor(par), dt,
                           setup_of(wl), torch.tensor(G))
    err = float((Gd.cpu() - gq).norm() / gq.norm())
    print("state bar rel err", err)
    assert err < 1e-11
    if par is not None:
        errp = float((pbar.cpu() - gp).norm() / gp.norm())
        print("param bar rel err", errp)
        assert errp < 1e-11
    st.close()


@pytest.mark.parametrize("pde,d,N,nc,R", [(inputs.ACOUSTIC, 3, 3, (2, 2, 3), 2),
                                          (inputs.ELASTIC, 2, 3, (3, 2), 3)])
def test_linear_vjp_other_picard_counts_and_no_material_bars(pde, d, N, nc, R):
    """Linear fluxes take the power-form adjoint for the default count R = N + 1
    and the stored-iterate adjoint otherwise: both against the oracle's
    autograd at the same R; without a material-bar buffer the state bar is
    unchanged (bitwise)."""
    wl = _wl(pde, d, N, nc).with_(picard_iters=R)
    Q = inputs.random_state(wl, seed=31, amplitude=0.05)
    par = inputs.cell_params(wl, seed=3)
    G = np.random.default_rng(9).standard_normal(Q.shape)
    dt = 2e-3
    print("case vjp R", pde, d, N, R, flush=True)
    gq, gp = oadj.step_vjp(torch.tensor(Q), torch.tensor(par), dt, setup_of(wl), torch.tensor(G))
    st = Stepper(wl, adjoint=True)
    Qd, pd = torch.tensor(Q, device="cuda"), torch.tensor(par, device="cuda")
    Gd = torch.tensor(G, device="cuda")
    pbar = torch.zeros_like(pd)
    st.step_adjoint(Qd, pd, st.scalar(dt), Gd, pbar)
    torch.cuda.synchronize()
    assert float((Gd.cpu() - gq).norm() / gq.norm()) < 1e-11
    assert float((pbar.cpu() - gp).norm() / gp.norm()) < 1e-11
    st.close()
    wl1 = wl.with_(picard_iters=0)
    gq1, _ = oadj.step_vjp(torch.tensor(Q), torch.tensor(par), dt, setup_of(wl1), torch.tensor(G))
    st = Stepper(wl1, adjoint=True)
    G1, G2 = torch.tensor(G, device="cuda"), torch.tensor(G, device="cuda")
    st.step_adjoint(Qd, pd, st.scalar(dt), G1, torch.zeros_like(pd))
    st.step_adjoint(Qd, pd, st.scalar(dt), G2, None)
    torch.cuda.synchronize()
    assert torch.equal(G1, G2)
    assert float((G1.cpu() - gq1).norm() / gq1.norm()) < 1e-11
    st.close()


def test_step_vjp_central_differences():
    """<dJ/dQ, v> against (J(Q + e v) - J(Q - e v)) / 2e for J = <G, S(Q)>,
    on 4 seeded directions (GPU forward only)."""
    wl = _wl(inputs.EULER, 3, 3, (3, 3, 2), (1.4,))
    Q = torch.tensor(inputs.random_state(wl, seed=90, amplitude=0.05), device="cuda")
    rng = np.random.default_rng(3)
    G = torch.tensor(rng.standard_normal(tuple(Q.shape)), device="cuda")
    st = Stepper(wl, adjoint=True)
    dtt = st.scalar(2e-3)

    def J(X):
        Y = X.clone()
        st.step(Y, None, dtt)
        return float((Y * G).sum())
    gb = G.clone()
    st.step_adjoint(Q, None, dtt, gb)
    for k in range(4):
        v = torch.tensor(rng.standard_normal(tuple(Q.shape)), device="cuda")
        eps = 1e-6 * float(Q.norm()) / float(v.norm())
        fd = (J(Q + eps * v) - J(Q - eps * v)) / (2 * eps)
        an = float((gb * v).sum())
        print("fd", fd, "adjoint", an)
        assert abs(fd - an) <= 1e-6 * abs(an)
    st.close()


def test_rollout_receiver_misfit_acoustics():
    """C4 reduced: acoustics N=3, 5^3 cells, per-cell sound speed, 12 steps,
    checkpoint every 5, 8 receivers; gradients of the misfit w.r.t. the
    initial pressure DoFs and the sound speed against the oracle's autograd,
    plus a central finite difference on the sound speed."""
    wl = inputs.preset("C4").with_(n_cells=(5, 5, 5))
    Q0 = inputs.initial_state(wl)
    c = inputs.cell_params(wl, seed=0)
    ctrue = inputs.cell_params(wl, seed=2)
    pts = inputs.receivers(8, 3, seed=1)
    dt = wl.cfl * wl.h / (3 * 7 * float(c.max()))
    steps = 12
    st = Stepper(wl, adjoint=True)
    rc, rr = receiver_rows(wl, pts)
    rec = (torch.tensor(rc, device="cuda"), torch.tensor(rr, device="cuda"))
    # synthetic data from the "true" sound speed (forward only)
    with torch.no_grad():
        _, data = rollout(st, torch.tensor(Q0, device="cuda"), torch.tensor(ctrue, device="cuda"),
                          steps, dt=dt, checkpoint_every=5, receivers=rec)
    Qg = torch.tensor(Q0, device="cuda", requires_grad=True)
    cg = torch.tensor(c, device="cuda", requires_grad=True)
    _, smp = rollout(st, Qg, cg, steps, dt=dt, checkpoint_every=5, receivers=rec)
    J = 0.5 * ((smp - data) ** 2).sum()
    J.backward()
    s = setup_of(wl)
    dts = [dt] * steps
    Jo, gq, gc = oadj.grad_misfit(torch.tensor(Q0), torch.tensor(c), s, dts, pts, data.detach().cpu())
    print("J gpu", float(J), "oracle", Jo)
    assert abs(float(J) - Jo) <= 1e-12 * abs(Jo)
    eq = float((Qg.grad[..., 0].cpu() - gq[..., 0]).norm() / gq[..., 0].norm())
    ec = float((cg.grad.cpu() - gc).norm() / gc.norm())
    print("grad rel err p0", eq, "c", ec)
    assert eq < 1e-10 and ec < 1e-10
    v = torch.tensor(np.random.default_rng(3).standard_normal(c.shape), device="cuda")
    eps = 1e-6

    def Jc(cc):
        with torch.no_grad():
            _, sm = rollout(st, torch.tensor(Q0, device="cuda"), cc, steps, dt=dt,
                            checkpoint_every=5, receivers=rec)
        return float(0.5 * ((sm - data) ** 2).sum())
    fd = (Jc(cg.detach() + eps * v) - Jc(cg.detach() - eps * v)) / (2 * eps)
    an = float((cg.grad * v).sum())
    print("fd", fd, "adjoint", an)
    assert abs(fd - an) <= 1e-6 * abs(an)
    st.close()


def test_rollout_final_kinetic_energy_euler():
    """C5 reduced: Euler N=3 on 4^3 cells, Fourier density, p = rho^gamma,
    6 steps with device-computed dt (recorded and held fixed), checkpoint
    every 4: dKE(Q_N)/dQ0 (density component) against the oracle."""
    wl = inputs.preset("C5").with_(order=3, n_cells=(4, 4, 4), length=4 / 48)
    Q0 = inputs.initial_state(wl, seed=0)
    st = Stepper(wl, adjoint=True)
    Qg = torch.tensor(Q0, device="cuda", requires_grad=True)
    z, om = np.polynomial.legendre.leggauss(wl.n)
    w1 = torch.tensor(0.5 * om, device="cuda")
    QN, _ = rollout(st, Qg, None, 6, cfl=wl.cfl, checkpoint_every=4)
    KE = kinetic_energy(QN, 3, wl.h, w1)
    KE.backward()
    # the same dt sequence for the oracle, read back from a forward-only pass
    Q = torch.tensor(Q0, device="cuda")
    dts = [float(x.item()) for x in st.run(Q, None, 6, cfl=wl.cfl, record_dt=True)]
    Jo, g = oadj.grad_final_ke(torch.tensor(Q0), setup_of(wl), dts)
    print("KE gpu", float(KE), "oracle", Jo)
    assert abs(float(KE) - Jo) <= 1e-10 * abs(Jo)
    err = float((Qg.grad[..., 0].cpu() - g[..., 0]).norm() / g[..., 0].norm())
    print("dKE/drho0 rel err", err)
    assert err < 1e-9
    st.close()


def test_rollout_final_kinetic_energy_euler_n7_fd():
    """C5 at its order: Euler N=7 (8^3 nodes per cell) on 2 x 2 x 1 cells, Fourier
    density with p = rho^gamma, 12 steps with the device-computed dt,
    checkpoint every 10 (two segments).  The gradient of the final kinetic
    energy w.r.t. the initial density DoFs is taken with the recorded dt
    sequence held fixed (the dependence of dt on the state through the wave
    speed maximum is not differentiated); against the oracle's autograd with
    the same dts, and against central differences of the GPU forward run
    with the same dts on 4 seeded directions and 8 sampled coordinates."""
    wl = inputs.preset("C5").with_(n_cells=(2, 2, 1), length=2 / 48)
    Q0 = inputs.initial_state(wl, seed=0)
    steps, k = 12, 10
    st = Stepper(wl, adjoint=True)
    z, om = np.polynomial.legendre.leggauss(wl.n)
    w1 = torch.tensor(0.5 * om, device="cuda")
    print("case C5 N=7 KE gradient", flush=True)
    Qg = torch.tensor(Q0, device="cuda", requires_grad=True)
    QN, _ = rollout(st, Qg, None, steps, cfl=wl.cfl, checkpoint_every=k)
    KE = kinetic_energy(QN, 3, wl.h, w1)
    KE.backward()
    g = Qg.grad[..., 0].detach()
    Q = torch.tensor(Q0, device="cuda")
    dts = [float(x.item()) for x in st.run(Q, None, steps, cfl=wl.cfl, record_dt=True)]
    Jo, go = oadj.grad_final_ke(torch.tensor(Q0), setup_of(wl), dts)
    print("KE gpu", float(KE), "oracle", Jo)
    assert abs(float(KE) - Jo) <= 1e-10 * abs(Jo)
    err = float((g.cpu() - go[..., 0]).norm() / go[..., 0].norm())
    print("dKE/drho0 rel err vs oracle", err)
    assert err < 1e-9

    dtd = [st.scalar(x) for x in dts]

    def J(X):
        Y = X.clone()
        for x in dtd:
            st.step(Y, None, x)
        return float(kinetic_energy(Y, 3, wl.h, w1))
    rng = np.random.default_rng(3)
    Q0d = torch.tensor(Q0, device="cuda")
    rho = Q0d[..., 0]
    gmax = float(g.abs().max())
    for kdir in range(4):
        v = torch.zeros_like(Q0d)
        v[..., 0] = torch.tensor(rng.standard_normal(tuple(rho.shape)), device="cuda")
        eps = 1e-6 * float(rho.norm()) / float(v.norm())
        fd = (J(Q0d + eps * v) - J(Q0d - eps * v)) / (2 * eps)
        an = float((g * v[..., 0]).sum())
        print("direction", kdir, "fd", fd, "adjoint", an)
        assert abs(fd - an) <= 1e-6 * abs(an)
    flat = rng.choice(rho.numel(), 8, replace=False)
    for f in flat:
        c_, a_ = divmod(int(f), rho.shape[1])
        v = torch.zeros_like(Q0d)
        v[c_, a_, 0] = 1.0
        eps = 1e-6 * float(rho.norm())
        fd = (J(Q0d + eps * v) - J(Q0d - eps * v)) / (2 * eps)
        an = float(g[c_, a_])
        print("coordinate", (c_, a_), "fd", fd, "adjoint", an)
        assert abs(fd - an) <= 1e-6 * max(abs(an), 1e-3 * gmax)
    st.close()


def test_rollout_receiver_misfit_fd_directions_and_coordinates():
    """C4 reduced (acoustics N=3, 5^3 cells, per-cell sound speed, 12 steps,
    checkpoint every 5, 8 receivers): the misfit gradient against central
    differences on 8 seeded directions in (initial pressure DoFs, sound
    speed) jointly and on 16 sampled coordinates (8 pressure DoFs, 8 cells'
    sound speeds), eps = 1e-6 |theta| / |v|; relative bar 1e-6 (coordinates
    whose gradient is below 1e-3 of the largest are held to 1e-6 of that)."""
    wl = inputs.preset("C4").with_(n_cells=(5, 5, 5))
    Q0 = torch.tensor(inputs.initial_state(wl), device="cuda")
    c = torch.tensor(inputs.cell_params(wl, seed=0), device="cuda")
    ctrue = torch.tensor(inputs.cell_params(wl, seed=2), device="cuda")
    pts = inputs.receivers(8, 3, seed=1)
    dt = wl.cfl * wl.h / (3 * 7 * float(c.max()))
    steps, k = 12, 5
    st = Stepper(wl, adjoint=True)
    rc, rr = receiver_rows(wl, pts)
    rec = (torch.tensor(rc, device="cuda"), torch.tensor(rr, device="cuda"))
    print("case C4 FD directions", flush=True)
    with torch.no_grad():
        _, data = rollout(st, Q0, ctrue, steps, dt=dt, checkpoint_every=k, receivers=rec)
    Qg, cg = Q0.clone().requires_grad_(True), c.clone().requires_grad_(True)
    _, smp = rollout(st, Qg, cg, steps, dt=dt, checkpoint_every=k, receivers=rec)
    (0.5 * ((smp - data) ** 2).sum()).backward()
    gp, gc = Qg.grad[..., 0].detach(), cg.grad.detach()

    def J(Qx, cx):
        with torch.no_grad():
            _, sm = rollout(st, Qx, cx, steps, dt=dt, checkpoint_every=k, receivers=rec)
        return float(0.5 * ((sm - data) ** 2).sum())
    p0 = Q0[..., 0]
    theta = float(torch.sqrt((p0 ** 2).sum() + (c ** 2).sum()))
    rng = np.random.default_rng(3)
    for kdir in range(8):
        vp = torch.tensor(rng.standard_normal(tuple(p0.shape)), device="cuda")
        vc = torch.tensor(rng.standard_normal(tuple(c.shape)), device="cuda")
        eps = 1e-6 * theta / float(torch.sqrt((vp ** 2).sum() + (vc ** 2).sum()))
        Qp, Qm = Q0.clone(), Q0.clone()
        Qp[..., 0] += eps * vp
        Qm[..., 0] -= eps * vp
        fd = (J(Qp, c + eps * vc) - J(Qm, c - eps * vc)) / (2 * eps)
        an = float((gp * vp).sum() + (gc * vc).sum())
        print("direction", kdir, "fd", fd, "adjoint", an)
        assert abs(fd - an) <= 1e-6 * abs(an)
    gpm, gcm = float(gp.abs().max()), float(gc.abs().max())
    for f in rng.choice(p0.numel(), 8, replace=False):
        c_, a_ = divmod(int(f), p0.shape[1])
        eps = 1e-6 * theta
        Qp, Qm = Q0.clone(), Q0.clone()
        Qp[c_, a_, 0] += eps
        Qm[c_, a_, 0] -= eps
        fd = (J(Qp, c) - J(Qm, c)) / (2 * eps)
        an = float(gp[c_, a_])
        print("pressure DoF", (c_, a_), "fd", fd, "adjoint", an)
        assert abs(fd - an) <= 1e-6 * max(abs(an), 1e-3 * gpm)
    for f in rng.choice(c.shape[0], 8, replace=False):
        eps = 1e-6 * theta
        cp_, cm_ = c.clone(), c.clone()
        cp_[int(f), 0] += eps
        cm_[int(f), 0] -= eps
        fd = (J(Q0, cp_) - J(Q0, cm_)) / (2 * eps)
        an = float(gc[int(f), 0])
        print("sound speed", int(f), "fd", fd, "adjoint", an)
        assert abs(fd - an) <= 1e-6 * max(abs(an), 1e-3 * gcm)
    st.close()


@pytest.mark.parametrize("order,cells,prec", [
    (3, (4, 4, 4), inputs.FP32),
    (3, (4, 4, 4), inputs.BF16),
    (7, (2, 2, 1), inputs.BF16),      # C5's order with the matrix-core predictor
])
def test_rollout_final_kinetic_energy_reduced_precision_forward(order, cells, prec):
    """C5 with its reduced-precision predictor: the forward steps (and the
    checkpoint recomputes) run with the float or bfloat16 predictor, and the
    float64 adjoint steps are applied at those states, so the gradient is the
    float64 linearisation of the step along the reduced-precision trajectory.
    Against the oracle's grad_final_ke_mixed (its mixed step and float64 step
    VJPs at the emulated states), 6 steps at a fixed dt, checkpoint every 4.
    Bars: the final KE within 8 u k of the emulation's (u = 2^-24, k steps:
    the float predictor's derived per-step state bound); the gradient's
    relative L2 distance from the emulation's within that same 8 u k for the
    float predictor (the reverse sweep maps a relative state change to a
    relative gradient change of the same order over these steps), and for
    bfloat16 within a tenth of the emulation's own distance from the float64
    gradient, so the GPU gradient follows the bfloat16 trajectory, not the
    float64 one."""
    wl = inputs.preset("C5").with_(order=order, n_cells=cells, length=cells[0] / 48)
    Q0 = inputs.initial_state(wl, seed=0)
    s = setup_of(wl)
    Qt = torch.tensor(Q0)
    dt = ostep.cfl_dt(ostep.max_wave_speed(Qt, None, s), wl.cfl, s)
    steps, k = 6, 4
    name = {inputs.FP32: "fp32", inputs.BF16: "bf16"}[prec]
    print(f"case reduced-precision forward KE gradient N={order} cells={cells} {name}", flush=True)
    st = Stepper(wl, adjoint=True)
    fw = Stepper(wl.with_(precision=prec))
    z, om = np.polynomial.legendre.leggauss(wl.n)
    w1 = torch.tensor(0.5 * om, device="cuda")
    Qg = torch.tensor(Q0, device="cuda", requires_grad=True)
    QN, _ = rollout(st, Qg, None, steps, dt=dt, checkpoint_every=k, forward=fw)
    KE = kinetic_energy(QN, 3, wl.h, w1)
    KE.backward()
    g = Qg.grad[..., 0].detach().cpu()
    st.close()
    fw.close()
    Je, ge = oadj.grad_final_ke_mixed(Qt, s, [dt] * steps, name)
    J64, g64 = oadj.grad_final_ke(Qt, s, [dt] * steps)
    ge, g64 = ge[..., 0], g64[..., 0]
    d_ge = float((g - ge).norm() / ge.norm())
    d_e64 = float((ge - g64).norm() / g64.norm())
    print("KE gpu", float(KE), "emulation", Je, "float64", J64,
          "| gradient rel L2: gpu vs emulation", d_ge, "emulation vs float64", d_e64, flush=True)
    bar = 8 * 2.0 ** -24 * steps
    assert abs(float(KE) - Je) <= bar * abs(Je)
    if prec == inputs.FP32:
        assert d_ge <= bar
    else:
        assert d_ge <= 0.1 * d_e64
