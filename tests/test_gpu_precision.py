"""The reduced-precision predictor against the oracle's precision emulation.

The oracle's mixed step (oracle/mixed.py) rounds exactly what the kernels
round: the Picard iteration in float32 (q, the fluxes, the contractions with
D against the pencil's reference flux, the time contraction with P), the
hull stored in float32, everything after it (time averages accumulated in
float64, volume term, Rusanov, face lift, update) in float64.  The GPU path
computes the same float32 quantities in a different order (and with FMA
contraction), so the two agree to float rounding, element by element.

Tolerance (derived, per step, element-wise):
  * every float32 value in the predictor carries at most a few units of
    roundoff u = 2^-24 of its size; the new iterate q = u - c P rhs is
    rounded at |q|, the hull traces once more when stored, so the traces of
    the two computations differ by at most about 4 u |q|, and likewise the
    flux traces by 4 u |F|;
  * the corrector turns a trace difference into an update difference
    through (dt/h) (LR + LL) (|dF|/2 + s |dq|/2), with (dt/h) s the Courant
    number (below 0.05 here), |F| <~ s |q|, and LR, LL <= 1/w_min
    (w_min the smallest Gauss-Legendre weight, 0.1 at n = 5, 0.05 at n = 8);
    the volume term adds (dt/h) |Kv| |dFbar|, smaller still;
  * so one step differs by at most 16 (dt/h) s u |q| / w_min <= 8 u max|Q|
    for the cases below (with the Courant number 0.05 and w_min >= 0.05 and
    at most twice that for the flux term), and k steps by k times that.
The stated bound is 8 u k max|Q|; the measured figures are printed.
"""

import numpy as np
import pytest
import torch

from oracle import mixed, step as ostep
from oracle.diagnostics import rel_l2
from paper_1801_08682_amd import inputs
from paper_1801_08682_amd.inputs import ACOUSTIC, ELASTIC, EULER
from tests.helpers import gpu_run, setup_of

pytestmark = pytest.mark.gpu
U32 = 2.0 ** -24


def _case(pde, dim, order, cells, prec):
    pp = (1.4,) if pde == EULER else ()
    h = 1.0 / 9.0
    wl = inputs.Workload(f"p{pde}{dim}{order}", pde, dim, order, tuple(cells),
                         cells[0] * h, pp, precision=prec)
    Q0 = inputs.random_state(wl, seed=80 + order, amplitude=0.05)
    par = inputs.cell_params(wl, seed=81)
    s = setup_of(wl)
    Qt = torch.tensor(Q0)
    pt = None if par is None else torch.tensor(par)
    # a fixed dt at half the stable Courant number of the order
    dt = ostep.cfl_dt(ostep.max_wave_speed(Qt, pt, s), 0.5 * inputs.stable_cfl(order), s)
    return wl, Q0, par, s, Qt, pt, dt


CASES = [
    (EULER, 3, 4, (4, 3, 3)),      # the headline kernel: all slices in one LDS buffer
    (EULER, 3, 5, (3, 2, 2)),
    (EULER, 3, 7, (2, 2, 2)),      # slices in two batches
    (EULER, 2, 3, (5, 3)),         # several cells per workgroup
    (ELASTIC, 3, 5, (3, 2, 2)),    # 16-byte quads, one buffer, materials
    (ACOUSTIC, 3, 3, (4, 3, 3)),   # 16-byte quads, two cells per workgroup
]


@pytest.mark.parametrize("pde,dim,order,cells", CASES)
def test_float_predictor_matches_emulation(pde, dim, order, cells):
    steps = 2
    wl, Q0, par, s, Qt, pt, dt = _case(pde, dim, order, cells, inputs.FP32)
    print("case fp32 emulation", pde, dim, order, cells, "dt", dt, flush=True)
    Qg, flag, _ = gpu_run(wl, Q0, par, steps, dt=dt)
    Qe = mixed.run_mixed(Qt, pt, s, steps, "fp32", [dt] * steps)
    Q64 = Qt
    for _ in range(steps):
        Q64 = ostep.step(Q64, pt, dt, s)
    assert flag == 0
    dev = float((Qg - Qe).abs().max())
    scale = float(Qe.abs().max())
    print("max |gpu - emulation| / max|Q|", dev / scale,
          "| per-field rel L2 gpu vs emulation", [f"{x:.2e}" for x in rel_l2(Qg, Qe, s)],
          "| emulation vs float64", [f"{x:.2e}" for x in rel_l2(Qe, Q64, s)])
    assert dev <= 8 * U32 * steps * scale


BF16_CASES = [
    (EULER, 3, 4, (4, 3, 3)),
    (EULER, 3, 3, (4, 3, 3)),      # two cells per workgroup
    (EULER, 3, 7, (2, 2, 2)),
    (ELASTIC, 3, 5, (3, 2, 2)),
    (ACOUSTIC, 3, 3, (4, 3, 3)),
]


@pytest.mark.parametrize("pde,dim,order,cells", BF16_CASES)
def test_bf16_predictor_matches_emulation(pde, dim, order, cells):
    """The bfloat16 predictor (flux differences rounded to bfloat16, D as a
    bfloat16 pair, float32 accumulation on the matrix cores) against the
    emulation's "bf16" mode.  Both round x = F - F_ref to bfloat16, but they
    compute x in float32 in different orders, so an x within float rounding
    of a bfloat16 rounding boundary may round to the neighbouring bfloat16
    value on one side only; such a flip moves one contraction input by one
    bfloat16 unit (2^-8 of it), the size of the bfloat16 effect at that one
    input.  Bars: per field, the GPU-emulation difference is at most 10% of
    the emulation's own distance from float64 (rel. L2), and element-wise at
    most that distance plus the float32 bound of the float predictor."""
    steps = 2
    wl, Q0, par, s, Qt, pt, dt = _case(pde, dim, order, cells, inputs.BF16)
    print("case bf16 emulation", pde, dim, order, cells, "dt", dt, flush=True)
    Qg, flag, _ = gpu_run(wl, Q0, par, steps, dt=dt)
    Qe = mixed.run_mixed(Qt, pt, s, steps, "bf16", [dt] * steps)
    Q64 = Qt
    for _ in range(steps):
        Q64 = ostep.step(Q64, pt, dt, s)
    assert flag == 0
    e_ge = rel_l2(Qg, Qe, s)
    e_e64 = rel_l2(Qe, Q64, s)
    dev = float((Qg - Qe).abs().max())
    gap = float((Qe - Q64).abs().max())
    scale = float(Qe.abs().max())
    print("max |gpu - emulation| / max|Q|", dev / scale, "| max |emulation - float64| / max|Q|",
          gap / scale,
          "| per-field rel L2 gpu vs emulation", [f"{x:.2e}" for x in e_ge],
          "| emulation vs float64", [f"{x:.2e}" for x in e_e64])
    assert bool((e_ge <= 0.1 * e_e64).all())
    assert dev <= gap + 8 * U32 * steps * scale
