"""GPU parity: the HIP path through the C ABI against the FP64 CPU oracle on
the same seeded inputs, element-wise (per-field relative L2, absolute where a
field's reference norm is negligible).  FP64 bar: 1e-12."""

import numpy as np
import pytest
import torch

from paper_1801_08682_amd import inputs
from tests.helpers import gpu_run, max_rel, oracle_run, per_field, setup_of

pytestmark = pytest.mark.gpu
TOL64 = 1e-12


def _wl(pde, dim, order, n_cells, pp=(), prec=inputs.FP64, R=0):
    h = 1.0 / 9.0
    return inputs.Workload(f"t{pde}{dim}{order}", pde, dim, order, tuple(n_cells),
                           n_cells[0] * h, tuple(pp), picard_iters=R, precision=prec)


def test_c1_full_parity_and_exact():
    """C1 at full size: 27x27 advection N=3, 10 steps, fixed dt."""
    wl = inputs.preset("C1")
    Q0 = inputs.initial_state(wl)
    dt = wl.cfl * wl.h / (wl.dim * (2 * wl.order + 1) * 1.0)
    print("case C1 dt", dt, flush=True)
    Qg, flag, _ = gpu_run(wl, Q0, None, wl.steps, dt=dt)
    Qo, _ = oracle_run(wl, Q0, None, wl.steps, dt=dt)
    assert flag == 0
    err = max_rel(Qg, Qo, wl)
    print("C1 rel L2 vs oracle", err)
    assert err < TOL64
    X = inputs.node_positions(wl)
    ex = np.sin(2 * np.pi * (X.sum(-1) - 1.5 * wl.steps * dt))[..., None]
    assert max_rel(Qg, torch.tensor(ex), wl) < 2e-6


@pytest.mark.parametrize("order", [0, 1, 2, 3, 4, 5])
def test_euler_2d_orders(order):
    wl = _wl(inputs.EULER, 2, order, (5, 3), (1.4,))
    Q0 = inputs.random_state(wl, seed=10 + order, amplitude=0.05)
    print("case euler2d N", order, flush=True)
    Qg, flag, dg = gpu_run(wl, Q0, None, 3, cfl=0.5, record_dt=True)
    Qo, do = oracle_run(wl, Q0, None, 3, cfl=0.5)
    assert flag == 0
    assert np.allclose(dg, do, rtol=1e-13, atol=0)
    assert max_rel(Qg, Qo, wl) < TOL64, per_field(Qg, Qo, wl)


@pytest.mark.parametrize("order", [1, 2, 3, 4, 5, 7])
def test_euler_3d_orders(order):
    """Ragged grid (cells not a multiple of any block size)."""
    wl = _wl(inputs.EULER, 3, order, (3, 2, 2) if order >= 5 else (5, 3, 2), (1.4,))
    Q0 = inputs.random_state(wl, seed=20 + order, amplitude=0.05)
    print("case euler3d N", order, flush=True)
    Qg, flag, dg = gpu_run(wl, Q0, None, 2, cfl=0.5, record_dt=True)
    Qo, do = oracle_run(wl, Q0, None, 2, cfl=0.5)
    assert flag == 0
    assert np.allclose(dg, do, rtol=1e-13, atol=0)
    assert max_rel(Qg, Qo, wl) < TOL64, per_field(Qg, Qo, wl)


@pytest.mark.parametrize("dim,order", [(2, 2), (2, 4), (3, 1), (3, 3), (3, 4), (3, 5)])
def test_acoustic(dim, order):
    wl = _wl(inputs.ACOUSTIC, dim, order, (4, 3, 2)[:dim])
    Q0 = inputs.random_state(wl, seed=30 + order)
    par = inputs.cell_params(wl, seed=0)
    print("case acoustic", dim, order, flush=True)
    Qg, flag, _ = gpu_run(wl, Q0, par, 2, dt=1e-3)
    Qo, _ = oracle_run(wl, Q0, par, 2, dt=1e-3)
    assert max_rel(Qg, Qo, wl) < TOL64, per_field(Qg, Qo, wl)


@pytest.mark.parametrize("dim,order", [(2, 1), (2, 3), (3, 2), (3, 4), (3, 5)])
def test_elastic(dim, order):
    wl = _wl(inputs.ELASTIC, dim, order, (3, 2, 2)[:dim])
    Q0 = inputs.random_state(wl, seed=40 + order)
    par = inputs.cell_params(wl, seed=0)
    print("case elastic", dim, order, flush=True)
    Qg, flag, _ = gpu_run(wl, Q0, par, 2, dt=1e-3)
    Qo, _ = oracle_run(wl, Q0, par, 2, dt=1e-3)
    assert max_rel(Qg, Qo, wl) < TOL64, per_field(Qg, Qo, wl)


@pytest.mark.parametrize("dim,order", [(2, 0), (2, 5), (3, 2), (3, 4)])
def test_advection(dim, order):
    wl = _wl(inputs.ADVECTION, dim, order, (4, 3, 2)[:dim], (1.0, -0.5, 0.25)[:dim])
    Q0 = inputs.random_state(wl, seed=50 + order)
    print("case advection", dim, order, flush=True)
    Qg, flag, _ = gpu_run(wl, Q0, None, 3, dt=2e-3)
    Qo, _ = oracle_run(wl, Q0, None, 3, dt=2e-3)
    assert max_rel(Qg, Qo, wl) < TOL64, per_field(Qg, Qo, wl)


def test_fp32_predictor_error_is_stated():
    """Mixed precision (float predictor, float64 corrector) against the FP64
    oracle: the error is small and far above FP64 round-off."""
    wl = _wl(inputs.EULER, 3, 4, (4, 3, 3), (1.4,), prec=inputs.FP32)
    Q0 = inputs.random_state(wl, seed=60)
    print("case fp32 euler3d", flush=True)
    Qg, flag, _ = gpu_run(wl, Q0, None, 2, dt=1e-3)
    Qo, _ = oracle_run(wl, Q0, None, 2, dt=1e-3)
    pf = per_field(Qg, Qo, wl)
    print("fp32 per-field rel L2", pf)
    assert max(pf) < 1e-5


@pytest.mark.parametrize("pde,dim,order,cells,pp", [
    (inputs.EULER, 3, 4, (1, 1, 1), (1.4,)),
    (inputs.EULER, 2, 3, (1, 4), (1.4,)),
    (inputs.EULER, 3, 7, (1, 2, 1), (1.4,)),
    (inputs.ELASTIC, 3, 2, (7, 1, 2), ()),
    (inputs.ACOUSTIC, 3, 3, (1, 2, 1), ()),
])
def test_single_cell_axes(pde, dim, order, cells, pp):
    """One cell along an axis: the periodic neighbour is the cell itself
    (a single cell is its own neighbour on every face)."""
    wl = _wl(pde, dim, order, cells, pp)
    Q0 = inputs.random_state(wl, seed=70 + order, amplitude=0.05)
    par = inputs.cell_params(wl, seed=71)
    print("case single-cell axes", pde, dim, order, cells, flush=True)
    Qg, flag, dg = gpu_run(wl, Q0, par, 3, cfl=0.5, record_dt=True)
    Qo, do = oracle_run(wl, Q0, par, 3, cfl=0.5)
    assert flag == 0
    assert np.allclose(dg, do, rtol=1e-13, atol=0)
    assert max_rel(Qg, Qo, wl) < TOL64, per_field(Qg, Qo, wl)


@pytest.mark.parametrize("prec", [inputs.FP64, inputs.FP32])
@pytest.mark.parametrize("order", [3, 4, 5, 7])
def test_uniform_flow_is_kept(order, prec):
    """A uniform moving state is an exact solution: the derivative of a
    constant flux must vanish in the predictor's own precision (the float
    predictor included), so the state after two steps differs from the
    initial one by float64 round-off only, not by float rounding."""
    wl = _wl(inputs.EULER, 3, order, (4, 3, 3), (1.4,), prec=prec)
    rho, u, p = 1.2, np.array([0.3, -0.2, 0.1]), 0.9
    q = np.concatenate([[rho], rho * u, [p / 0.4 + 0.5 * rho * u @ u]])
    Q0 = np.broadcast_to(q, (wl.ncells, wl.n ** 3, 5)).copy()
    print("case uniform flow N", order, "prec", prec, flush=True)
    Qg, flag, _ = gpu_run(wl, Q0, None, 2, cfl=0.5)
    assert flag == 0
    dev = float(np.abs(Qg.numpy() - Q0).max())
    print("max deviation", dev)
    assert dev < 1e-13


def test_c2_full_size_sampled_parity():
    """C2 at full size (81^3, N=4) in the bench's launch configuration: one
    step on the GPU; 24 sampled cells (corners, edges, bump centre, random)
    recomputed by the oracle cell by cell; plus conservation over the grid."""
    from oracle import step as ostep
    from oracle.diagnostics import totals
    wl = inputs.preset("C2")
    Q0 = inputs.initial_state(wl)
    s = setup_of(wl)
    lam = ostep.max_wave_speed(torch.tensor(Q0[::97]), None, s)
    print("case C2 full one step", flush=True)
    from paper_1801_08682_amd.stepper import Stepper
    st = Stepper(wl)
    Q = torch.tensor(Q0, device="cuda")
    lamd = st.scalar()
    dtd = st.scalar()
    st.wave_speed(Q, None)
    st.cfl_dt(wl.cfl, lamd, dtd)
    flag = torch.zeros(1, dtype=torch.int32, device="cuda")
    st.step(Q, None, dtd, flag)
    torch.cuda.synchronize()
    dt = float(dtd.item())
    assert abs(float(lamd.item()) - ostep.max_wave_speed(torch.tensor(Q0), None, s)) < 1e-14
    assert int(flag.item()) == 0
    rng = np.random.default_rng(0)
    nc = 81
    c = lambda x, y, z: x + nc * (y + nc * z)
    cells = [c(0, 0, 0), c(80, 80, 80), c(40, 40, 40), c(0, 40, 80), c(80, 0, 40),
             c(39, 40, 41), c(40, 41, 40)] + list(rng.integers(0, nc ** 3, 17))
    ref = ostep.step_cells(torch.tensor(Q0), None, dt, s, cells)
    got = Q[torch.tensor(cells, device="cuda")].cpu()
    err = (got - ref).abs().max() / ref.abs().max()
    print("C2 sampled max rel err", float(err))
    assert float(err) < 1e-13
    M0 = totals(torch.tensor(Q0), s)
    M1 = totals(Q.cpu(), s)
    assert float((M1 - M0).abs().max()) < 1e-13 * float(M0.abs().max())
    st.close()


class _Rows:
    """Rows of a device tensor fetched on demand: the oracle's sampled step
    indexes the state by cell, so only the sampled cells and their face
    neighbours leave the GPU."""

    def __init__(self, t):
        self.t = t

    def __getitem__(self, idx):
        return self.t[torch.as_tensor(idx).to(self.t.device)].cpu()


def test_c2_moving_flow_sampled_parity_10_steps():
    """C2's grid and launch configuration (81^3, N = 4) on a moving flow
    (8 seeded Fourier density modes, p = rho^gamma: acoustic waves, all five
    fields change): 10 steps with dt recomputed on the device from each new
    state.  After every step, 6 sampled cells are recomputed by the oracle
    from the GPU's previous state (its sampled one-step evaluation), and the
    error is stated per field relative to that cell's update Q1 - Q0 (not to
    the state), so the bar applies to the change a step makes.  The last
    state's wave-speed maximum is checked against the oracle's over the whole
    grid.  Bars: the largest error over the sampled cells is at most 1e-13
    of the largest state value, and per field at most 1e-9 of the largest
    update of that field.  The update-relative bar cannot be 1e-12: a step
    changes the state by 1e-4 to 1e-3 of its size here (and density and
    energy by O(dt^2) in the first step, which starts at rest), and the
    update is formed from O(1) values, so float64 rounding of the state
    alone (a few ulp) is 1e-12 to 1e-10 of the update (measured: at most
    1.8e-10, and 4.6e-16 of the state)."""
    from oracle import step as ostep
    from paper_1801_08682_amd.stepper import Stepper
    wl = inputs.preset("C2").with_(extra={"ic": "fourier"})
    s = setup_of(wl)
    Q0 = inputs.initial_state(wl, seed=0)
    print("case C2 moving flow, 10 steps", flush=True)
    st = Stepper(wl)
    Q = torch.tensor(Q0, device="cuda")
    del Q0
    dtd, lamd = st.scalar(), st.scalar()
    flag = torch.zeros(1, dtype=torch.int32, device="cuda")
    st.wave_speed(Q, None)
    st.cfl_dt(wl.cfl, None, dtd)
    rng = np.random.default_rng(5)
    worst_upd, worst_state = 0.0, 0.0
    for k in range(10):
        Qprev = Q.clone()
        dt = float(dtd.item())
        st.step(Q, None, dtd, flag)
        st.cfl_dt(wl.cfl, lamd, dtd)
        torch.cuda.synchronize()
        cells = list(rng.integers(0, wl.ncells, 6))
        ref = ostep.step_cells(_Rows(Qprev), None, dt, s, cells)
        idx = torch.tensor(cells, device="cuda")
        got, prev = Q[idx].cpu(), Qprev[idx].cpu()
        err = (got - ref).abs().amax(dim=(0, 1))
        upd = (ref - prev).abs().amax(dim=(0, 1))
        e_upd = float((err / upd).max())
        e_state = float(err.max() / ref.abs().max())
        print(f"step {k}: dt {dt:.6e} max err / update per field {e_upd:.3e}, / state "
              f"{e_state:.3e}", flush=True)
        worst_upd, worst_state = max(worst_upd, e_upd), max(worst_state, e_state)
        del Qprev
    assert int(flag.item()) == 0
    Qc = Q.cpu()
    lam_o = ostep.max_wave_speed(Qc, None, s)
    assert abs(float(lamd.item()) - lam_o) <= 1e-14 * lam_o
    st.close()
    assert worst_state < 1e-13
    assert worst_upd < 1e-9


def test_bitwise_determinism_and_flag():
    """Run-to-run bitwise determinism (no float atomics), and the
    admissibility flag for a negative density."""
    wl = _wl(inputs.EULER, 3, 3, (6, 5, 4), (1.4,))
    Q0 = inputs.random_state(wl, seed=70, amplitude=0.05)
    a, fa, _ = gpu_run(wl, Q0, None, 3, dt=1e-3)
    b, fb, _ = gpu_run(wl, Q0, None, 3, dt=1e-3)
    assert torch.equal(a, b) and fa == 0 and fb == 0
    Qbad = Q0.copy()
    Qbad[7, :, 0] = -0.5
    _, fbad, _ = gpu_run(wl, Qbad, None, 1, dt=1e-4)
    assert fbad & 2


@pytest.mark.parametrize("name", ["C3", "C4", "C5"])
def test_full_size_sampled_parity(name):
    """C3 (elasticity N=5, 64^3), C4 (acoustics N=3, 48^3) and C5 (Euler N=7,
    48^3) at full size, float64: one step; 12 sampled cells (corners, centre,
    random) recomputed by the oracle cell by cell; conservation over the grid."""
    from oracle import step as ostep
    from oracle.diagnostics import totals
    from paper_1801_08682_amd.stepper import Stepper
    wl = inputs.preset(name)
    Q0 = inputs.initial_state(wl, seed=0)
    par = inputs.cell_params(wl, seed=0)
    s = setup_of(wl)
    print("case full", name, flush=True)
    st = Stepper(wl)
    Q = torch.tensor(Q0, device="cuda")
    pd = None if par is None else torch.tensor(par, device="cuda")
    dtd = st.scalar()
    st.wave_speed(Q, pd)
    st.cfl_dt(wl.cfl, None, dtd)
    st.step(Q, pd, dtd)
    torch.cuda.synchronize()
    dt = float(dtd.item())
    nc = wl.n_cells[0]
    c = lambda x, y, z: x + nc * (y + nc * z)
    rng = np.random.default_rng(1)
    cells = [c(0, 0, 0), c(nc - 1, nc - 1, nc - 1), c(nc // 2, nc // 2, nc // 2)] + \
        list(rng.integers(0, nc ** 3, 9))
    ref = ostep.step_cells(torch.tensor(Q0), None if par is None else torch.tensor(par), dt, s, cells)
    got = Q[torch.tensor(cells, device="cuda")].cpu()
    err = float((got - ref).abs().max() / ref.abs().max())
    print(name, "sampled max rel err", err)
    assert err < 1e-12
    M0, M1 = totals(torch.tensor(Q0), s), totals(Q.cpu(), s)
    assert float((M1 - M0).abs().max()) < 1e-12 * (1.0 + float(M0.abs().max()))
    st.close()
