"""Benchmark: DoF-updates/s of the ADER-DG step on 3D Euler N=4, 81^3 cells.

One "step" = the whole hot path on one batch: the space-time predictor,
extrapolation and volume term, the Rusanov solves, face lift and update, the
wave speeds and the device-side time step.  ``value`` times the paper's
shifted, fused and optimistic stepping (Alg. 2; adg_fused_begin / one
adg_fused_sweep per step / adg_fused_end): each sweep corrects step k and
predicts step k+1 in one kernel, with dt = 0.99 x the admissible step under
the creeping average and a device-side predictor rerun when a new state does
not admit the dt already used.  The two-kernel Alg. 1 path (adg_predict,
adg_correct, adg_cfl_dt) is timed too and reported under ``two_kernel``.

Workload: 3D compressible Euler, gamma = 1.4, N = 4 (5^3 Gauss-Legendre nodes
per cell), 81^3 periodic cells on [0,1]^3, density 1 + 0.1 exp(-r^2/0.02),
u = 0, p = 1, Rusanov flux, admissible dt = 0.5625 h / (3 (2N+1) lambda_max)
(0.9 of the measured linear-stability limit of the N = 4 step).  Inputs are
synthetic and resident in HBM before the timed region.

Prints ONE JSON line.  Besides the float64 path it times the mixed-precision
path (float predictor, float64 corrector) on the same workload and reports
its per-field relative L2 difference to the float64 path after the same
number of steps.
"""

import argparse
import ctypes
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "DoF-updates/s, 3D Euler N=4: FP64 vs mixed-precision at stated L2 error"
FP64_PEAK_TFLOPS = 78.6      # 256 CU x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz
HBM_PEAK_GBPS = 8000.0
FP32_PEAK_TFLOPS = 157.3     # published vector fp32 (packed); this path issues unpacked FMAs
C_DT = 0.99                  # security factor of the optimistic time step (the paper's value)


def pred_flops_per_cell(d, n, m, R, cF):
    """Algorithmic flops of one adg_predict per cell (sum-factorised method):
    R Picard iterations [d+1 contractions of n x n along one axis over the
    m n^(d+1) space-time values, d fluxes at n^(d+1) nodes, axis sums and the
    update], then the final fluxes, time averages, volume contraction,
    face extrapolations and Q~ = u + dt V."""
    pic = 2 * (d + 1) * m * n ** (d + 2) + cF * n ** (d + 1) + (d + 2) * m * n ** (d + 1)
    fin = (cF * n ** (d + 1) + 2 * (d + 1) * m * n ** (d + 1) + 2 * d * m * n ** (d + 1)
           + 8 * d * m * n ** d + 2 * m * n ** d)
    return R * pic + fin


def corr_flops_per_cell(d, n, m):
    """Algorithmic flops of the corrector per cell: Rusanov on the 2d faces
    (n^(d-1) nodes, about 5m + 15 flops each incl. the wave speeds), the
    face lift, the update and the wave speeds of the new state."""
    return 2 * d * n ** (d - 1) * (5 * m + 15) + 4 * d * m * n ** d + 2 * m * n ** d + 15 * n ** d


def step_flops_per_cell(d, n, m, R, cF=30):
    """Algorithmic flops of one whole step per cell: predictor + corrector
    (c_F = 30 flops for the three 3D Euler fluxes at a node)."""
    return pred_flops_per_cell(d, n, m, R, cF) + corr_flops_per_cell(d, n, m)


def cpu_model():
    """The host CPU's model name (as lscpu prints it)."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def corr_bytes_per_cell(d, n, m, real_bytes):
    """Algorithmic HBM bytes of one adg_correct per cell: read Q~ and write Q
    (2 m n^d float64) and read the face hull once (2d faces x 2 quantities x
    m n^(d-1) values); a neighbour's traces re-read from HBM are waste."""
    return 2 * m * n ** d * 8 + 2 * d * 2 * m * n ** (d - 1) * real_bytes


def measured_traffic(key):
    """Calibrated rocprofv3 FETCH_SIZE + WRITE_SIZE bytes per launch recorded
    in profiles/, valid only while the kernel sources hash the same."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "hbm_traffic_euler3d_n4_81cubed.json")
    try:
        rec = json.load(open(path))
    except (OSError, ValueError):
        return None
    h = hashlib.sha256()
    for f in rec["kernel_sources"]:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    if h.hexdigest() != rec["source_sha256"] or key not in rec:
        return None
    return rec[key]["hbm_bytes"]


def cpu_baseline(args):
    """The oracle, untuned, on a bounded sample of the same workload."""
    import torch
    from oracle import step as ostep
    from paper_1801_08682_amd import inputs
    k = args.cpu_cells
    wl = inputs.Workload("sample", inputs.EULER, 3, 4, (k, k, k), k / 81.0, (1.4,),
                         extra={"ic": "bump"})
    Q = torch.tensor(inputs.initial_state(wl))
    s = ostep.Setup(wl.pde, 3, 4, wl.n_cells, wl.h, wl.pde_param)
    dt = ostep.cfl_dt(ostep.max_wave_speed(Q, None, s), inputs.stable_cfl(4), s)
    Q = ostep.step(Q, None, dt, s)               # warm-up
    t0 = time.perf_counter()
    for _ in range(args.cpu_steps):
        dt = ostep.cfl_dt(ostep.max_wave_speed(Q, None, s), inputs.stable_cfl(4), s)
        Q = ostep.step(Q, None, dt, s)
    t = time.perf_counter() - t0
    return {"value": wl.ncells * wl.dofs_per_cell * args.cpu_steps / t,
            "unit": "DoF-updates/s", "cores": torch.get_num_threads(), "kind": "oracle",
            "sample": f"{k}^3-cell periodic grid of the same workload (Euler N=4, "
                      f"h=1/81, bump), {args.cpu_steps} steps after 1 warm-up, "
                      f"torch CPU float64", "cpu_model": cpu_model()}


def adjoint_bench(args):
    """C4 at full size: 3D acoustics N=3, 48^3 cells, per-cell sound speed,
    200 steps, receiver misfit at 64 receivers, gradient by the checkpointed
    rollout (adg_step forward, adg_step_adjoint backward, checkpoint every 20)."""
    import torch
    from paper_1801_08682_amd import inputs
    from paper_1801_08682_amd.rollout import rollout, receiver_rows
    from paper_1801_08682_amd.stepper import Stepper
    wl = inputs.preset("C4")
    steps, k = args.adj_steps, wl.extra["checkpoint"]
    Q0 = torch.tensor(inputs.initial_state(wl), device="cuda")
    c = torch.tensor(inputs.cell_params(wl, seed=0), device="cuda")
    ctrue = torch.tensor(inputs.cell_params(wl, seed=2), device="cuda")
    rc, rr = receiver_rows(wl, inputs.receivers(64, 3, seed=1))
    rec = (torch.tensor(rc, device="cuda"), torch.tensor(rr, device="cuda"))
    dt = wl.cfl * wl.h / (3 * (2 * wl.order + 1) * float(c.max()))
    st = Stepper(wl, adjoint=True)
    with torch.no_grad():
        _, data = rollout(st, Q0, ctrue, steps, dt=dt, checkpoint_every=k, receivers=rec)
    # untimed warm-up of the backward path over one checkpoint interval
    torch.cuda.empty_cache()
    Qw, cw = Q0.clone().requires_grad_(True), c.clone().requires_grad_(True)
    _, smp = rollout(st, Qw, cw, k, dt=dt, checkpoint_every=k, receivers=rec)
    (0.5 * ((smp - data[:k]) ** 2).sum()).backward()
    del Qw, cw, smp
    Q = Q0.clone()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st.run(Q, c, steps, dt=dt)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    Qg = Q0.clone().requires_grad_(True)
    cg = c.clone().requires_grad_(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, smp = rollout(st, Qg, cg, steps, dt=dt, checkpoint_every=k, receivers=rec)
    J = 0.5 * ((smp - data) ** 2).sum()
    J.backward()
    torch.cuda.synchronize()
    t_fb = time.perf_counter() - t0
    # one adg_step_adjoint against one adg_step, both alone on the device
    Qs, Gs, pb = Q0.clone(), torch.randn_like(Q0), torch.zeros_like(c)
    dts = st.scalar(dt)
    reps = 20
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    st.step_adjoint(Qs, c, dts, Gs, pb)
    torch.cuda.synchronize()
    ev[0].record()
    for _ in range(reps):
        st.step(Qs, c, dts)
    ev[1].record()
    for _ in range(reps):
        st.step_adjoint(Qs, c, dts, Gs, pb)
    ev[2].record()
    torch.cuda.synchronize()
    fwd_ms, adj_ms = ev[0].elapsed_time(ev[1]) / reps, ev[1].elapsed_time(ev[2]) / reps
    st.close()
    return {"workload": f"3D acoustics N=3, 48^3 cells, {steps} steps, 64 receivers, "
                        f"checkpoint every {k}", "forward_s": t_fwd,
            "forward_plus_backward_s": t_fb, "ratio": t_fb / t_fwd, "J": float(J.detach()),
            "step_ms": fwd_ms, "adjoint_step_ms": adj_ms, "step_ratio": adj_ms / fwd_ms,
            "grad_norm_p0": float(Qg.grad[..., 0].norm()), "grad_norm_c": float(cg.grad.norm())}


def c5_gradient_bench(args):
    """C5 at full size: 3D Euler N=7, 48^3 cells, Fourier density, 50 steps
    with the device-computed dt (recorded, then held fixed in the reverse
    sweep), gradient of the final kinetic energy w.r.t. the initial density
    DoFs by the checkpointed rollout (checkpoint every 10).  float64 forward
    and adjoint; also one adg_step_adjoint against one adg_step; then the
    same gradient with the forward steps taken by the float and by the
    bfloat16 (matrix-core) predictor and the float64 adjoint at their states,
    with its distance from the float64 gradient."""
    import numpy as np
    import torch
    from paper_1801_08682_amd import inputs
    from paper_1801_08682_amd.rollout import kinetic_energy, rollout
    from paper_1801_08682_amd.stepper import Stepper
    wl = inputs.preset("C5")
    steps, k = args.adj_steps if args.adj_steps != 200 else wl.steps, wl.extra["checkpoint"]
    Q0 = torch.tensor(inputs.initial_state(wl, seed=0), device="cuda")
    z, om = np.polynomial.legendre.leggauss(wl.n)
    w1 = torch.tensor(0.5 * om, device="cuda")
    st = Stepper(wl, adjoint=True)
    # untimed warm-up of the backward path over one checkpoint interval
    Qw = Q0.clone().requires_grad_(True)
    QN, _ = rollout(st, Qw, None, k, cfl=wl.cfl, checkpoint_every=k)
    kinetic_energy(QN, 3, wl.h, w1).backward()
    del Qw, QN
    Q = Q0.clone()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st.run(Q, None, steps, cfl=wl.cfl)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    Qg = Q0.clone().requires_grad_(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    QN, _ = rollout(st, Qg, None, steps, cfl=wl.cfl, checkpoint_every=k)
    KE = kinetic_energy(QN, 3, wl.h, w1)
    KE.backward()
    torch.cuda.synchronize()
    t_fb = time.perf_counter() - t0
    g = Qg.grad[..., 0]
    Qs, Gs = Q0.clone(), torch.randn_like(Q0)
    dts = st.scalar(wl.cfl * wl.h / (3 * (2 * wl.order + 1) * 2.0))
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    st.step_adjoint(Qs, None, dts, Gs, None)
    torch.cuda.synchronize()
    reps = 5
    ev[0].record()
    for _ in range(reps):
        st.step(Qs, None, dts)
    ev[1].record()
    for _ in range(reps):
        st.step_adjoint(Qs, None, dts, Gs, None)
    ev[2].record()
    torch.cuda.synchronize()
    fwd_ms, adj_ms = ev[0].elapsed_time(ev[1]) / reps, ev[1].elapsed_time(ev[2]) / reps
    out = {"workload": f"3D Euler N=7, 48^3 cells, {steps} steps, final kinetic energy, "
                       f"checkpoint every {k}", "forward_s": t_fwd, "forward_plus_backward_s": t_fb,
           "ratio": t_fb / t_fwd, "KE": float(KE.detach()), "grad_norm_rho0": float(g.norm()),
           "step_ms": fwd_ms, "adjoint_step_ms": adj_ms, "step_ratio": adj_ms / fwd_ms}
    # the configured form: the forward steps (and the checkpoint recomputes)
    # with the reduced-precision predictor, the float64 adjoint at their states
    g64 = g.detach().clone()
    for name, prec in (("fp32_forward", inputs.FP32), ("bf16_forward", inputs.BF16)):
        fw = Stepper(wl.with_(precision=prec))
        Q = Q0.clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fw.run(Q, None, steps, cfl=wl.cfl)
        torch.cuda.synchronize()
        tf = time.perf_counter() - t0
        Qg = Q0.clone().requires_grad_(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        QN, _ = rollout(st, Qg, None, steps, cfl=wl.cfl, checkpoint_every=k, forward=fw)
        KEm = kinetic_energy(QN, 3, wl.h, w1)
        KEm.backward()
        torch.cuda.synchronize()
        tfb = time.perf_counter() - t0
        gm = Qg.grad[..., 0]
        out[name] = {"forward_s": tf, "forward_plus_backward_s": tfb, "KE": float(KEm.detach()),
                     "KE_rel_vs_fp64": float(KEm.detach()) / float(KE.detach()) - 1.0,
                     "grad_rel_l2_vs_fp64": float((gm - g64).norm() / g64.norm())}
        fw.close()
        del Qg, QN
    st.close()
    return out


def other_workload(args, torch):
    """One line for a non-headline workload: float64 and float-predictor
    throughput over its step count and the float path's per-field L2
    difference to the float64 path at the end."""
    from paper_1801_08682_amd import inputs
    from paper_1801_08682_amd.stepper import Stepper
    wl = inputs.preset(args.workload)
    steps = wl.steps if args.steps == 100 else args.steps
    Q0 = torch.tensor(inputs.initial_state(wl, seed=0), device="cuda")
    par = inputs.cell_params(wl, seed=0)
    par = None if par is None else torch.tensor(par, device="cuda")
    res, states = {}, {}
    from paper_1801_08682_amd import _lib
    precs = [inputs.FP64, inputs.FP32]
    try:
        _lib.query(_lib.make_config(wl.dim, wl.order, wl.n_cells, [wl.length] * wl.dim, wl.pde,
                                    wl.pde_param, precision=inputs.BF16))
        precs.append(inputs.BF16)
    except _lib.AdgError:
        pass
    for prec in precs:
        st = Stepper(wl.with_(precision=prec))
        if wl.adaptive_dt:
            lam = None
            cfl, dt = wl.cfl, None
        else:
            speed = 1.0 if wl.pde == inputs.ADVECTION else float(
                (par[:, 0] if wl.pde == inputs.ACOUSTIC else
                 torch.sqrt((par[:, 1] + 2 * par[:, 2]) / par[:, 0])).max())
            cfl, dt = None, wl.cfl * wl.h / (wl.dim * (2 * wl.order + 1) * speed)
        Q = Q0.clone()
        st.run(Q, par, 2, cfl=cfl, dt=dt)          # warm-up on a copy
        Q = Q0.clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st.run(Q, par, steps, cfl=cfl, dt=dt)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        res[prec] = {"value": wl.ncells * wl.dofs_per_cell * steps / wall,
                     "ms_per_step": wall * 1e3 / steps}
        states[prec] = Q
        st.close()
    n = wl.n
    z, om = np.polynomial.legendre.leggauss(n)
    w = torch.tensor(0.5 * om, device="cuda")
    W = w
    for _ in range(wl.dim - 1):
        W = torch.kron(w, W)
    ref = states[inputs.FP64]
    norms = [float(torch.sqrt((W * ref[..., v] ** 2).sum())) for v in range(wl.m)]

    def errs(got):
        err = []
        for v in range(wl.m):
            e = float(torch.sqrt((W * (got[..., v] - ref[..., v]) ** 2).sum()))
            err.append(e / norms[v] if norms[v] > 1e-8 * max(norms) else e)
        return err
    out = {"metric": "DoF-updates/s", "unit": "DoF-updates/s", "workload": wl.name,
           "config": {"pde": wl.pde, "dim": wl.dim, "order": wl.order, "cells": wl.ncells,
                      "steps": steps, "cfl": wl.cfl},
           "fp64": res[inputs.FP64], "fp32_predictor": res[inputs.FP32],
           "fp32_rel_l2_vs_fp64_per_field": errs(states[inputs.FP32])}
    if inputs.BF16 in res:
        out["bf16_predictor"] = res[inputs.BF16]
        out["bf16_rel_l2_vs_fp64_per_field"] = errs(states[inputs.BF16])
    return out


def run_path(st, Q0, steps, warmup, cfl, torch):
    """Warm-up on a copy, then `steps` timed steps; per-kernel event times."""
    Q = Q0.clone()
    dtt = st.scalar()
    st.wave_speed(Q, None)
    st.cfl_dt(cfl, None, dtt)
    for _ in range(warmup):
        st.step(Q, None, dtt)
        st.cfl_dt(cfl, None, dtt)
    Q.copy_(Q0)
    st.wave_speed(Q, None)
    st.cfl_dt(cfl, None, dtt)
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(steps)]
    stream = st.stream
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    with torch.cuda.stream(stream):
        for k in range(steps):
            ev[k][0].record(stream)
            st.predict(Q, None, dtt)
            ev[k][1].record(stream)
            st.correct(Q, None, dtt)
            ev[k][2].record(stream)
            st.cfl_dt(cfl, None, dtt)
            ev[k][3].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    pred = sum(e[0].elapsed_time(e[1]) for e in ev) / steps
    corr = sum(e[1].elapsed_time(e[2]) for e in ev) / steps
    dtk = sum(e[2].elapsed_time(e[3]) for e in ev) / steps
    return Q, wall, pred, corr, dtk


def spacetime_workload(args, torch):
    """A workload with space-time traces (Table 1's cardinalities: q and F.n
    at every time node of every face node, a Rusanov solve per time node):
    fused and two-kernel paths with the float64 and the float predictor, and
    the float64 corrector's bandwidth against its algorithmic bytes.  C2
    takes --cells; C5 runs at its own size."""
    from paper_1801_08682_amd import inputs
    from paper_1801_08682_amd.stepper import Stepper
    name = args.workload if args.workload in ("C2", "C5") else "C2"
    wl = inputs.preset(name)
    if name == "C2":
        wl = wl.with_(n_cells=(args.cells,) * 3, length=args.cells / 81.0)
    d, n, m = wl.dim, wl.n, wl.m
    Q0 = torch.tensor(inputs.initial_state(wl), device="cuda")
    dofs = wl.ncells * wl.dofs_per_cell
    out = {"metric": "DoF-updates/s", "unit": "DoF-updates/s",
           "workload": f"{name} with space-time traces ({wl.n_cells[0]}^3 cells, Euler N={wl.order})"}
    for key, prec, size in (("fp64", inputs.FP64, 8), ("fp32_predictor", inputs.FP32, 4)):
        st = Stepper(wl.with_(precision=prec), fused=True, spacetime=True)
        Q, wall, sweep, reruns, _ = run_fused_path(st, Q0, args.steps, args.warmup, wl.cfl, C_DT, torch)
        _, wall2, pred, corr, dtk = run_path(st, Q0, args.steps, args.warmup, wl.cfl, torch)
        st.close()
        hull = 2 * d * 2 * m * n ** d * size              # bytes per cell, every time node
        leg = {"fused": {"value": dofs * args.steps / wall, "ms_per_step": wall * 1e3 / args.steps,
                         "sweep_ms": sweep, "reruns": reruns},
               "two_kernel": {"value": dofs * args.steps / wall2,
                              "ms_per_step": wall2 * 1e3 / args.steps,
                              "kernel_ms": {"predict": pred, "correct": corr, "cfl_dt": dtk}},
               "hull_bytes_per_cell": hull,
               "correct_hbm_GBps": (2 * m * n ** d * 8 + hull) * wl.ncells / (corr * 1e-3) / 1e9}
        if key == "fp64":
            out.update(leg)
        else:
            out[key] = leg
    return out


def run_fused_path(st, Q0, steps, warmup, cfl, c_dt, torch):
    """Alg. 2 stepping: warm-up run on a copy, then adg_fused_begin, `steps`
    - 1 sweeps (each timed with events on the stepper's stream) and
    adg_fused_end, all inside the timed region."""
    Q = Q0.clone()
    st.run_fused(Q, None, warmup + 1, cfl, c_dt)
    Q.copy_(Q0)
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(2)] for _ in range(steps - 1)]
    stream = st.stream
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    with torch.cuda.stream(stream):
        dt_used, reruns = st.fused_begin(Q, None, cfl, c_dt, True, steps)
        for k in range(steps - 1):
            ev[k][0].record(stream)
            st.fused_sweep()
            ev[k][1].record(stream)
        st.fused_end()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    sweep = sum(e[0].elapsed_time(e[1]) for e in ev) / max(steps - 1, 1)
    return Q, wall, sweep, int(reruns.item()), dt_used


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cells", type=int, default=81)
    ap.add_argument("--cpu-cells", type=int, default=15)
    ap.add_argument("--cpu-steps", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-peaks", action="store_true")
    ap.add_argument("--adjoint-only", action="store_true",
                    help="print only the C4 adjoint rollout's line")
    ap.add_argument("--c5-gradient", action="store_true",
                    help="print only the C5 kinetic-energy gradient rollout's line")
    ap.add_argument("--adj-steps", type=int, default=200)
    ap.add_argument("--workload", default="C2", choices=["C1", "C2", "C3", "C4", "C5"],
                    help="C2 is the headline line; the others print their own line "
                         "(float64 and float-predictor throughput and per-field error)")
    ap.add_argument("--traces", default="time-integrated", choices=["time-integrated", "spacetime"],
                    help="spacetime: print one line for C2 (or --workload C5) with space-time "
                         "traces and a Rusanov solve per time node, float64 and float predictor")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32", "bf16"],
                    help="predictor precision of the headline line (fp64 is the metric's "
                         "float64 step; the others are for profiling the reduced-precision "
                         "kernels alone, with --no-mixed)")
    ap.add_argument("--acc-steps", type=int, default=100,
                    help="steps after which the reduced-precision error is stated (the metric's "
                         "100; smaller only to shorten profiled runs)")
    ap.add_argument("--copy-calib-mb", type=int, default=0,
                    help="also run a plain device copy of this many MiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only; multi-GPU sharding is "
              "described in DESIGN.md but not implemented.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1801_08682_amd import inputs
    from paper_1801_08682_amd.stepper import Stepper

    if args.c5_gradient:
        print(json.dumps(c5_gradient_bench(args)), flush=True)
        return
    if args.adjoint_only:
        res = adjoint_bench(args)
        if args.copy_calib_mb:
            res["copy_calib_bytes"] = copy_calibration(args, torch)
        print(json.dumps(res), flush=True)
        return
    if args.traces == "spacetime" and args.workload in ("C2", "C5"):
        res = spacetime_workload(args, torch)
        if args.copy_calib_mb:
            res["copy_calib_bytes"] = copy_calibration(args, torch)
        print(json.dumps(res), flush=True)
        return
    if args.workload != "C2":
        print(json.dumps(other_workload(args, torch)), flush=True)
        return
    wl = inputs.preset("C2").with_(n_cells=(args.cells,) * 3,
                                   length=args.cells / 81.0)
    d, n, m = wl.dim, wl.n, wl.m
    print(f"[bench] building inputs {wl.n_cells} N={wl.order}", file=sys.stderr, flush=True)
    Q0 = torch.tensor(inputs.initial_state(wl), device="cuda")
    dofs = wl.ncells * wl.dofs_per_cell
    R = wl.order + 1
    fpc = pred_flops_per_cell(d, n, m, R, 30)
    fsc = step_flops_per_cell(d, n, m, R, 30)
    hull = 2 * d * 2 * m * n ** (d - 1)                      # hull doubles per cell
    full = args.cells == 81
    prec = {"fp64": inputs.FP64, "fp32": inputs.FP32, "bf16": inputs.BF16}[args.precision]
    st = Stepper(wl.with_(precision=prec), fused=True)
    print("[bench] fp64 fused run", file=sys.stderr, flush=True)
    Q64, wall, sweep, reruns, dts = run_fused_path(st, Q0, args.steps, args.warmup, wl.cfl,
                                                   C_DT, torch)
    print("[bench] fp64 two-kernel run", file=sys.stderr, flush=True)
    _, wall2, pred, corr, dtk = run_path(st, Q0, args.steps, args.warmup, wl.cfl, torch)
    st.close()
    del st
    achieved = fsc * wl.ncells / (sweep * 1e-3) / 1e12
    pred_achieved = fpc * wl.ncells / (pred * 1e-3) / 1e12
    out = {
        "metric": METRIC, "value": dofs * args.steps / wall, "unit": "DoF-updates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32", "bf16": "bf16+f32"}[args.precision],
        "data": "synthetic",
        "config": {"workload": f"3D compressible Euler N=4, {args.cells}^3 periodic cells "
                               "on [0,1]^3, Gaussian density bump, Rusanov, adaptive dt: "
                               f"{C_DT} x 0.5625 h/(3 (2N+1) lambda_max) with the creeping "
                               "average and device-side reruns (shifted, fused, optimistic "
                               "stepping, Alg. 2; 0.5625 = 0.9 of the N=4 stability limit)",
                   "cells": wl.ncells, "dofs_per_cell": wl.dofs_per_cell,
                   "picard_iters": R, "precision": args.precision, "stepping": "fused (Alg. 2)"},
        "kernel_ms": {"sweep": sweep},
        "reruns": reruns,
        "dt_first_last": [float(dts[0]), float(dts[args.steps - 1])],
        "cell_updates_per_s": wl.ncells * args.steps / wall,
        "legendre_point_updates_per_s": wl.ncells * n ** d * args.steps / wall,
        "roofline": {"kernel": "k_fused (adg_fused_sweep: corrector of step k + predictor of "
                               "step k+1)", "bound": "alu", "achieved": achieved,
                     "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP64_PEAK_TFLOPS,
                     "hbm_frac": wl.ncells * (2 * wl.dofs_per_cell * 8 + 2 * hull * 8)
                                 / (sweep * 1e-3) / (HBM_PEAK_GBPS * 1e9),
                     "binding": "alu (FP64 VALU and LDS; hbm_frac is far lower)",
                     "traffic": measured_traffic("k_fused_fp64") if full and prec == 0 else None,
                     "traffic_unit": "bytes per launch",
                     "algorithmic_bytes": wl.ncells * (2 * wl.dofs_per_cell * 8 + 2 * hull * 8),
                     "flops_per_cell": fsc,
                     "note": "achieved = algorithmic flops of the whole step per cell "
                             "(sum-factorised predictor with R = N+1 Picard iterations, "
                             "c_F = 30 flops for the three fluxes at a node, plus the "
                             "corrector) x cells / the sweep's event time (k_fused plus the "
                             "dt reduction and the skipped rerun launch)"},
        "two_kernel": {
            "stepping": "Alg. 1: adg_predict, adg_correct, adg_cfl_dt per step, dt = 0.5625 "
                        "h/(3 (2N+1) lambda_max)",
            "value": dofs * args.steps / wall2, "ms_per_step": wall2 * 1e3 / args.steps,
            "kernel_ms": {"predict": pred, "correct": corr, "cfl_dt": dtk},
            "predict_roofline": {"kernel": "k_pred (adg_predict)", "bound": "alu",
                                 "achieved": pred_achieved, "peak": FP64_PEAK_TFLOPS,
                                 "unit": "TFLOP/s", "frac": pred_achieved / FP64_PEAK_TFLOPS,
                                 "traffic": measured_traffic("k_pred_fp64") if full and prec == 0 else None,
                                 "algorithmic_bytes": wl.ncells * (wl.dofs_per_cell * 8 * 2
                                                                   + hull * 8)},
            "correct_hbm": {"achieved_GBps": corr_bytes_per_cell(d, n, m, 8) * wl.ncells
                            / (corr * 1e-3) / 1e9, "peak_GBps": 8000.0,
                            "algorithmic_bytes": corr_bytes_per_cell(d, n, m, 8) * wl.ncells,
                            "traffic": measured_traffic("k_corr_fp64") if full and prec == 0 else None}},
    }
    if not args.no_mixed:
        out.update(mixed_paths(args, wl, Q0, dofs, torch))
    if not args.no_adjoint:
        print("[bench] adjoint (C4 misfit gradient)", file=sys.stderr, flush=True)
        out["adjoint"] = adjoint_bench(args)
    if args.copy_calib_mb:
        out["copy_calib_bytes"] = copy_calibration(args, torch)
    if not args.no_peaks:
        print("[bench] measured peaks", file=sys.stderr, flush=True)
        mp = measured_peaks(torch)
        out["measured_peaks"] = mp
        out["roofline"]["frac_of_measured_peak"] = achieved / mp["fp64_fma_TFLOPs"]
        out["two_kernel"]["correct_hbm"]["frac_of_measured_copy"] = (
            out["two_kernel"]["correct_hbm"]["achieved_GBps"] / mp["hbm_copy_GBps"])
    if not args.no_cpu:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(args)
    print(json.dumps(out), flush=True)


ACC_STEPS = 100     # the metric states the reduced-precision error at step 100


def mixed_paths(args, wl, Q0, dofs, torch):
    """The reduced-precision predictors (float: float32 Picard iteration;
    bf16: float32 with the pencil contractions on the matrix cores, inputs
    rounded to bfloat16, float32 accumulation) with the float64 corrector:
    timed like the float64 path, and their per-field relative L2 difference
    to the float64 path after ACC_STEPS fused steps (untimed, whatever
    --steps is), on the headline state and on a moving flow."""
    from paper_1801_08682_amd import inputs
    from paper_1801_08682_amd.stepper import Stepper
    n, m = wl.n, wl.m
    W = torch.tensor(np.kron(np.kron(st32_w(n), st32_w(n)), st32_w(n)), device="cuda")
    wlf = wl.with_(extra={"ic": "fourier"})
    Qf = torch.tensor(inputs.initial_state(wlf), device="cuda")
    inits = {"bump": Q0, "moving_flow": Qf}

    acc = args.acc_steps

    def run100(prec, Qi):
        st = Stepper(wl.with_(precision=prec), fused=True)
        Q = Qi.clone()
        st.run_fused(Q, None, acc, wl.cfl, C_DT)
        torch.cuda.synchronize()
        st.close()
        return Q

    print("[bench] float64 reference states at step 100", file=sys.stderr, flush=True)
    ref = {k: run100(inputs.FP64, Qi) for k, Qi in inits.items()}
    res = {}
    for prec, key, desc in ((inputs.FP32, "mixed", "fp32 predictor, fp64 corrector"),
                            (inputs.BF16, "mixed_bf16",
                             "bf16-input matrix-core contractions with fp32 accumulation in "
                             "an fp32 predictor, fp64 corrector")):
        print(f"[bench] {key} runs", file=sys.stderr, flush=True)
        st = Stepper(wl.with_(precision=prec), fused=True)
        _, wall, sweep, reruns, _ = run_fused_path(st, Q0, args.steps, args.warmup, wl.cfl,
                                                   C_DT, torch)
        _, wallb, pred, corr, dtk = run_path(st, Q0, args.steps, args.warmup, wl.cfl, torch)
        st.close()
        errs = {k: field_errors(run100(prec, Qi), ref[k], W, m, torch) for k, Qi in inits.items()}
        res[key] = {"precision": desc,
                    "value": dofs * args.steps / wall, "ms_per_step": wall * 1e3 / args.steps,
                    "kernel_ms": {"sweep": sweep}, "reruns": reruns,
                    "two_kernel": {"value": dofs * args.steps / wallb,
                                   "ms_per_step": wallb * 1e3 / args.steps,
                                   "kernel_ms": {"predict": pred, "correct": corr,
                                                 "cfl_dt": dtk}},
                    "rel_l2_vs_fp64_per_field": errs["bump"],
                    "rel_l2_vs_fp64_per_field_moving_flow": errs["moving_flow"],
                    "l2_step": acc,
                    "l2_note": f"per-field relative L2 (Gauss-Legendre weights) after "
                               f"{acc} fused steps of each path against the float64 GPU "
                               "path (itself checked against the oracle step by step on this "
                               "grid); absolute L2 for fields with negligible norm (momentum "
                               "of the bump); the bump is a stationary contact, the moving "
                               "flow is 8 seeded Fourier density modes with p = rho^gamma on "
                               "the same grid"}
    del ref, inits, Qf
    return res


def copy_calibration(args, torch):
    """Three plain device copies of a known size, for scaling the HBM
    counters of a profiled run."""
    nbytes = args.copy_calib_mb << 20
    src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    return nbytes


def measured_peaks(torch):
    """Achievable rates on this device for the two resources that bound the
    step: vector FMA throughput (16 independent chains per thread, 16384
    workgroups of 256) and streaming HBM bandwidth (copy and triad over
    2 GiB arrays); best of 5 event-timed launches each."""
    from paper_1801_08682_amd import _lib
    P = _lib.load_peaks()
    stream = torch.cuda.current_stream()
    h = ctypes.c_void_p(stream.cuda_stream)

    def best(launch, reps=5):
        launch()                                   # warm-up
        ts = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            launch()
            e1.record(stream)
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1) * 1e-3)
        return min(ts)

    out = {}
    blocks, iters = 16384, 12500          # rates still rise up to about 8192 workgroups
    sink = torch.empty(blocks * 256, dtype=torch.float64, device="cuda")
    for prec, name in ((0, "fp64"), (1, "fp32_nonpacked")):
        def fma():
            assert P.adg_peak_fma(prec, blocks, iters, ctypes.c_void_p(sink.data_ptr()), h) == 0
        t = best(fma)
        out[f"{name}_fma_TFLOPs"] = blocks * 256 * 16 * iters * 2 / t / 1e12
        # the same rate with 1, 2, 3 and 4 waves per SIMD (256-thread workgroups,
        # one to four per CU): float FMAs of two waves issue together, float64
        # FMAs do not, so the float rate needs at least two waves with VALU work
        by = {}
        for w in (1, 2, 3, 4):
            nb, it = 256 * w, 6000
            def fma_w():
                assert P.adg_peak_fma(prec, nb, it, ctypes.c_void_p(sink.data_ptr()), h) == 0
            by[str(w)] = nb * 256 * 16 * it * 2 / best(fma_w, reps=3) / 1e12
        out[f"{name}_fma_TFLOPs_by_waves_per_simd"] = by
    n = 1 << 28
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.full((n,), 2.0, dtype=torch.float64, device="cuda")
    c = torch.empty_like(a)
    def copy():
        assert P.adg_stream_copy(ctypes.c_void_p(a.data_ptr()), ctypes.c_void_p(c.data_ptr()), n, h) == 0
    def triad():
        assert P.adg_stream_triad(ctypes.c_void_p(a.data_ptr()), ctypes.c_void_p(b.data_ptr()),
                                  ctypes.c_void_p(c.data_ptr()), 0.5, n, h) == 0
    out["hbm_copy_GBps"] = 16 * n / best(copy) / 1e9
    out["hbm_triad_GBps"] = 24 * n / best(triad) / 1e9
    assert float(c[-1]) == 2.0 and float(c[0]) == 2.0
    del a, b, c, sink
    out["note"] = ("published: FP64 vector 78.6 TFLOP/s, FP32 vector 157.3 TFLOP/s, HBM "
                   "8000 GB/s; the float kernel uses non-packed FMA (packed FP32 instructions are "
                   "not used in this build)")
    return out


def field_errors(Qa, Qb, W, m, torch):
    """Per-field relative L2 (quadrature weights W) of Qa against Qb; absolute
    L2 for a field whose norm is negligible next to the density's."""
    err = []
    r0 = float(torch.sqrt((W * Qb[..., 0] ** 2).sum()))
    for v in range(m):
        e = float(torch.sqrt((W * (Qa[..., v] - Qb[..., v]) ** 2).sum()))
        r = float(torch.sqrt((W * Qb[..., v] ** 2).sum()))
        err.append(e / r if r > 1e-8 * r0 else e)
    return err


def st32_w(n):
    z, om = np.polynomial.legendre.leggauss(n)
    return 0.5 * om


if __name__ == "__main__":
    main()
