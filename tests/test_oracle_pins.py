"""Pins of the FP64 oracle to things other than itself (CPU only).

Each test names what fixes the expected value: closed forms, textbook
schemes, exact polynomial algebra (numpy.polynomial, not the oracle's
barycentric tables), invariants, or values printed in the paper.
"""

import itertools
import math
import os

import numpy as np
import pytest
import torch
from numpy.polynomial import Polynomial as Poly

from oracle import step as ostep
from oracle.diagnostics import totals, l2, kinetic_energy, node_weights, point_values
from oracle.pde import make_pde, EULER, ACOUSTIC, ELASTIC, ADVECTION
from oracle.tables import make_tables
from paper_1801_08682_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def lagrange_polys(xi):
    """phi_j as numpy polynomials built from their roots (independent of the
    oracle's barycentric evaluation)."""
    out = []
    for j in range(len(xi)):
        p = Poly([1.0])
        for k in range(len(xi)):
            if k != j:
                p = p * Poly([-xi[k], 1.0]) / (xi[j] - xi[k])
        out.append(p)
    return out


def integ01(p):
    P = p.integ()
    return P(1.0) - P(0.0)


# ---------------------------------------------------------------- P1-P3 tables
@pytest.mark.parametrize("N", range(0, 9))
def test_gl_quadrature_exactness(N):
    """P1: GL with n = N+1 points integrates x^k exactly for k <= 2N+1; for
    x^(2n) the error is the closed-form Gauss remainder
    (n!)^4 / ((2n+1) ((2n)!)^2) on [0, 1]; nodes are symmetric."""
    t = make_tables(N)
    for k in range(2 * N + 2):
        assert abs((t.w * t.xi ** k).sum() - 1.0 / (k + 1)) < 1e-14
    n = N + 1
    k = 2 * n
    err = 1.0 / (k + 1) - (t.w * t.xi ** k).sum()
    exact = math.factorial(n) ** 4 / ((2 * n + 1) * math.factorial(2 * n) ** 2)
    assert abs(err - exact) < 1e-6 * exact + 1e-15
    assert np.allclose(t.xi + t.xi[::-1], 1.0, atol=1e-14)


@pytest.mark.parametrize("N", range(1, 9))
def test_derivative_matrix(N):
    """P2: D differentiates every polynomial of degree <= N exactly; D is
    nilpotent (D^(N+1) = 0) and annihilates constants."""
    t = make_tables(N)
    for k in range(N + 1):
        assert np.allclose(t.D @ t.xi ** k, k * t.xi ** max(k - 1, 0) if k else 0.0,
                           atol=1e-11 * 4 ** N)
    assert np.abs(np.linalg.matrix_power(t.D, N + 1)).max() < 1e-8 * 10 ** N
    assert np.abs(t.D.sum(1)).max() < 1e-12 * 4 ** N


@pytest.mark.parametrize("N", range(0, 9))
def test_time_and_face_operators(N):
    """P3: face values reproduce monomials at 0 and 1; K1 applied to ones is
    FL; P applied to tau^(k-1)/(k-1)! gives tau^k/k! for k <= N (the
    time-DG solution of z' = g, z(0) = 0 is exact on polynomials); lifting
    and volume operators satisfy sum_j w_j D[j][a] = FR_a - FL_a."""
    t = make_tables(N)
    for k in range(N + 1):
        assert abs(t.FL @ t.xi ** k - (1.0 if k == 0 else 0.0)) < 1e-12
        assert abs(t.FR @ t.xi ** k - 1.0) < 1e-12 * 4 ** N
    assert np.allclose(t.K1 @ np.ones(N + 1), t.FL, atol=1e-12 * 4 ** N)
    g = np.ones(N + 1)
    for k in range(1, N + 1):
        z = t.P @ g
        assert np.allclose(z, t.xi ** k / math.factorial(k), atol=1e-12 * 4 ** N)
        g = z
    assert np.allclose((t.w[:, None] * t.D).sum(0), t.FR - t.FL, atol=1e-12 * 4 ** N)
    # lifting: w * LL = FL, volume: w_a Kv[a][j] = w_j D[j][a]
    assert np.allclose(t.w * t.LL, t.FL) and np.allclose(t.w * t.LR, t.FR)


def test_tables_against_exact_polynomial_algebra():
    """P3: D, FL, FR, K1 from exact calculus on root-built Lagrange
    polynomials (no barycentric formula, no quadrature)."""
    for N in (2, 3, 5):
        t = make_tables(N)
        phi = lagrange_polys(t.xi)
        D = np.array([[phi[j].deriv()(x) for j in range(N + 1)] for x in t.xi])
        assert np.allclose(D, t.D, atol=1e-10)
        assert np.allclose([p(0.0) for p in phi], t.FL, atol=1e-12)
        assert np.allclose([p(1.0) for p in phi], t.FR, atol=1e-12)
        K1 = np.array([[phi[k](1) * phi[l](1) - integ01(phi[k].deriv() * phi[l])
                        for l in range(N + 1)] for k in range(N + 1)])
        assert np.allclose(K1, t.K1, atol=1e-10)
        M = np.array([[integ01(phi[a] * phi[b]) for b in range(N + 1)] for a in range(N + 1)])
        assert np.allclose(M, np.diag(t.w), atol=1e-10)


# ---------------------------------------------------------------- P4 predictor
def _poly_field(d, N, rng):
    """Random polynomial of degree <= N per axis: coefficient tensor c[k_0..]."""
    return rng.standard_normal((N + 1,) * d)


def _eval_poly(c, X):
    d = c.ndim
    out = np.zeros(X.shape[:-1])
    for idx in itertools.product(*[range(s) for s in c.shape]):
        term = c[idx]
        for i in range(d):
            term = term * X[..., i] ** idx[i]
        out = out + term
    return out


def _adv_apply(c, a):
    """Coefficients of (a . grad) p (exact polynomial algebra)."""
    d = c.ndim
    out = np.zeros_like(c)
    for i in range(d):
        dc = np.zeros_like(c)
        for k in range(1, c.shape[i]):
            src = [slice(None)] * d
            dst = [slice(None)] * d
            src[i] = k
            dst[i] = k - 1
            dc[tuple(dst)] += k * c[tuple(src)]
        out += a[i] * dc
    return out


@pytest.mark.parametrize("d,N", [(2, 3), (3, 2), (2, 5)])
def test_predictor_taylor_closed_form(d, N):
    """P4: for linear advection the r-th Picard iterate at the space-time
    nodes equals the Taylor polynomial sum_{k<=r} (-tau dt)^k/k! (a.grad)^k u
    for r <= N (exact algebra on monomial coefficients)."""
    rng = np.random.default_rng(1)
    a = np.array([1.0, -0.7, 0.4])[:d]
    h = 0.5
    s = ostep.Setup(ADVECTION, d, N, (1,) * d, h, tuple(a))
    c = _poly_field(d, N, rng)
    # node coordinates in the reference cell (scaled by h: x = h xi)
    t = s.tab
    grids = np.meshgrid(*([t.xi] * d), indexing="ij")
    Xi = np.stack([grids[d - 1 - i] for i in range(d)], -1)   # (..., k_{d-1}..k_0, d) x fastest last
    X = Xi * h
    u = torch.tensor(_eval_poly(c, X))[None, ..., None]
    dt = 0.3
    for r in range(1, N + 1):
        q = ostep.predictor(u, None, dt, s, iters=r)[0, ..., 0].numpy()
        ref = np.zeros_like(q)
        ck = c.copy()
        for k in range(r + 1):
            vals = _eval_poly(ck, X)
            for l in range(N + 1):
                ref[l] += (-t.xi[l] * dt) ** k / math.factorial(k) * vals
            ck = _adv_apply(ck, a)
        assert np.abs(q - ref).max() < 1e-11 * np.abs(ref).max(), r


@pytest.mark.parametrize("d,N", [(2, 3), (3, 2)])
def test_picard_exact_termination(d, N):
    """P4 / exact termination: for linear flux the Picard update vanishes at
    iteration N+1 for data varying along one axis, and at d*N+1 (not earlier)
    for general data, since the mixed derivatives survive up to total order dN."""
    rng = np.random.default_rng(2)
    s = ostep.Setup(ADVECTION, d, N, (1,) * d, 0.5, (1.0, 0.6, -0.3)[:d])
    n = N + 1
    gen = torch.tensor(rng.standard_normal((1,) + (n,) * d + (1,)))
    one_axis = gen.clone()
    one_axis[...] = gen.select(1, 0).unsqueeze(1) if d == 2 else gen[:, :1, :1]
    def upd(u, r):
        return float((ostep.predictor(u, None, 0.2, s, iters=r)
                      - ostep.predictor(u, None, 0.2, s, iters=r - 1)).abs().max())
    assert upd(one_axis, N + 1) < 1e-14
    assert upd(gen, d * N + 1) < 1e-14
    assert upd(gen, d * N) > 1e-8


# ------------------------------------------------------- P5 weak-form residual
def _lagrange_product_form(xi, x):
    """phi_b(x) and phi_b'(x) from the product formula (not the barycentric
    form the oracle uses); x is an array of points."""
    n = len(xi)
    V = np.ones((len(x), n))
    dV = np.zeros((len(x), n))
    for b in range(n):
        for k in range(n):
            if k != b:
                V[:, b] *= (x - xi[k]) / (xi[b] - xi[k])
        for j in range(n):
            if j == b:
                continue
            t = np.full(len(x), 1.0 / (xi[b] - xi[j]))
            for k in range(n):
                if k != b and k != j:
                    t *= (x - xi[k]) / (xi[b] - xi[k])
            dV[:, b] += t
    return V, dV


def _galerkin_1d(xi, nq=24):
    """Mass Mm[a][b] = int phi_a phi_b, Gd[a][b] = int phi_a phi_b' on [0, 1]
    and phi(0), by a 24-point Gauss rule (exact for these degrees) applied to
    the product-form basis."""
    z, om = np.polynomial.legendre.leggauss(nq)
    x, w = 0.5 * (1.0 + z), 0.5 * om
    V, dV = _lagrange_product_form(xi, x)
    return (V * w[:, None]).T @ V, (V * w[:, None]).T @ dV, _lagrange_product_form(xi, np.zeros(1))[0][0]


def _along(M, x, ax):
    return np.moveaxis(np.tensordot(M, x, axes=([1], [ax])), 0, ax)


def _weak_form_residual(q, u, F, dt, h, Mm, Gd, th0, flux_sign=1.0):
    """Residual of Eq. (3) for one cell, tested with theta_k(tau) phi_a(x),
    with the cell state u as the upwind value at tau = 0 and the collocated
    flux values F_i (reading R4), in the form
      int theta_k phi_a (dq/dtau + (dt/h) sum_i dF_i/dxi_i) + theta_k(0) int phi_a (q(0) - u).
    q, F_i: (t, k_{d-1}, .., k_0, m); u: (k_{d-1}, .., k_0, m)."""
    d = u.ndim - 1
    def kron(mats, X):          # mats[0] along time, mats[1 + a] along tensor axis 1 + a
        for ax, M in enumerate(mats):
            X = _along(M, X, ax)
        return X
    r = kron([Gd] + [Mm] * d, q)
    for i in range(d):                       # spatial axis i sits at tensor axis d - i
        mats = [Mm] + [Mm] * d
        mats[d - i] = Gd
        r = r + flux_sign * (dt / h) * kron(mats, F[i])
    q0 = np.tensordot(th0, q, axes=([0], [0]))
    r = r + th0.reshape((-1,) + (1,) * (d + 1)) * kron([Mm] * d, q0 - u)[None]
    return r


@pytest.mark.parametrize("d,N", [(2, 2), (3, 4), (3, 7)])
def test_converged_predictor_solves_space_time_weak_form(d, N):
    """P5: the converged Picard solution (Euler; 2D N=2 and one 3D cell at the
    headline order N=4 and at N=7) satisfies the cell-local space-time weak
    form of Eq. (3) with upwind initial data and collocated fluxes, evaluated
    with the product-form Lagrange basis and a 24-point Gauss rule.  A flipped
    flux sign leaves a residual of the size of the flux terms."""
    n = N + 1
    nc = (1,) * d
    s = ostep.Setup(EULER, d, N, nc, 0.2, (1.4,))
    wl = inputs.Workload("p5", inputs.EULER, d, N, nc, 0.2, (1.4,))
    u = torch.tensor(inputs.random_state(wl, seed=3, amplitude=0.2)).reshape(1, *([n] * d), d + 2)
    dt = 0.05 if d == 2 else (0.01 if N < 7 else 0.002)
    q = ostep.predictor(u, None, dt, s, tol=1e-16, max_iters=400)[0]
    Mm, Gd, th0 = _galerkin_1d(s.tab.xi)
    F = [s.pde.flux(q, i, None).numpy() for i in range(d)]
    r = _weak_form_residual(q.numpy(), u[0].numpy(), F, dt, s.h, Mm, Gd, th0)
    assert np.abs(r).max() < 1e-13
    bad = _weak_form_residual(q.numpy(), u[0].numpy(), F, dt, s.h, Mm, Gd, th0, flux_sign=-1.0)
    assert np.abs(bad).max() > 1e-5


# ----------------------------------------------------- P6, P7 invariants
def _rand_case(pde, d, N, nc, seed, amp=0.05):
    h = 1.0 / 7.0
    pp = {EULER: (1.4,), ADVECTION: (1.0, -0.5, 0.3)[:d]}.get(pde, ())
    wl = inputs.Workload("r", pde, d, N, nc, nc[0] * h, pp)
    Q = torch.tensor(inputs.random_state(wl, seed=seed, amplitude=amp))
    par = inputs.cell_params(wl, seed=seed)
    par = None if par is None else torch.tensor(par)
    return ostep.Setup(pde, d, N, nc, h, pp), Q, par


@pytest.mark.parametrize("pde", [ADVECTION, EULER, ACOUSTIC, ELASTIC])
@pytest.mark.parametrize("d", [2, 3])
def test_constant_state_preserved(pde, d):
    """P6: a constant state is a steady solution of every PDE; the step keeps
    it to round-off (uniform material)."""
    N = 3 if d == 2 else 2
    s, Q, par = _rand_case(pde, d, N, (3, 2, 2)[:d], 4)
    const = Q[0, 0].clone()
    Qc = const.expand_as(Q).clone()
    if par is not None:
        par = par[0:1].expand_as(par).clone()
    out = ostep.step(Qc, par, 0.01, s)
    assert (out - Qc).abs().max() < 1e-13 * (1 + const.abs().max())


@pytest.mark.parametrize("pde", [ADVECTION, EULER, ACOUSTIC, ELASTIC])
@pytest.mark.parametrize("d", [2, 3])
def test_conservation(pde, d):
    """P7: sum of h^d W_a Q over the periodic domain is conserved to
    round-off, also with per-cell materials: the volume term has zero cell
    integral (rows of D sum to zero) and each face flux is shared by its two
    cells, so the face terms telescope."""
    N = 3 if d == 2 else 2
    s, Q, par = _rand_case(pde, d, N, (4, 3, 2)[:d], 5)
    M0 = totals(Q, s)
    out = ostep.step(Q, par, 0.01, s)
    assert (totals(out, s) - M0).abs().max() < 1e-14 * (1 + M0.abs().max())


@pytest.mark.parametrize("pde", [ACOUSTIC, ELASTIC])
def test_conservation_uniform_material(pde):
    s, Q, par = _rand_case(pde, 3, 2, (3, 2, 2), 6)
    par = par[0:1].expand_as(par).clone()
    M0 = totals(Q, s)
    out = ostep.step(Q, par, 0.01, s)
    assert (totals(out, s) - M0).abs().max() < 1e-14 * (1 + M0.abs().max())


# ------------------------------------------------------------ P8 N = 0 is FV
@pytest.mark.parametrize("pde", [EULER, ACOUSTIC])
def test_order_zero_is_first_order_fv_rusanov(pde):
    """P8: with N = 0 the step is the textbook first-order finite-volume
    scheme with the Rusanov flux (App. A, Corollary 8), written out here."""
    d = 2
    s, Q, par = _rand_case(pde, d, 0, (5, 4), 7, amp=0.1)
    dt = 0.01
    out = ostep.step(Q, par, dt, s)
    nx, ny = s.n_cells
    U = Q[:, 0, :].reshape(ny, nx, -1)
    P = None if par is None else par.reshape(ny, nx, -1)
    pde_ = s.pde
    ref = U.clone()
    for i, ax in ((0, 1), (1, 0)):
        UR = torch.roll(U, -1, dims=ax)
        PR = None if P is None else torch.roll(P, -1, dims=ax)
        fL = pde_.flux(U, i, P)
        fR = pde_.flux(UR, i, PR)
        sp = torch.maximum(pde_.speed(U, i, P), pde_.speed(UR, i, PR))[..., None]
        Fh = 0.5 * (fL + fR) - 0.5 * sp * (UR - U)           # flux at i+1/2
        ref = ref - dt / s.h * (Fh - torch.roll(Fh, 1, dims=ax))
    assert (out.reshape(ny, nx, -1) - ref).abs().max() < 1e-14


# ----------------------------------------------------- P9 accuracy, C1 exact
def test_c1_sine_convergence():
    """P9: C1 (advection of sin(2 pi (x + y)) with a = (1, 0.5), N = 3) against
    the exact solution sin(2 pi (x + y - 1.5 t)): order >= N + 1 - 0.3 from
    9^2 to 81^2 cells at a fixed final time."""
    errs = []
    T = 9 * 0.9 * (1.0 / 27) / 14.0
    for nc in (9, 27, 81):
        wl = inputs.preset("C1").with_(n_cells=(nc, nc))
        s = ostep.Setup(wl.pde, 2, 3, wl.n_cells, wl.h, wl.pde_param)
        dt = 0.9 * wl.h / (7 * 2 * 1.0)
        steps = int(round(T / dt))
        Q, _ = ostep.run(torch.tensor(inputs.initial_state(wl)), None, s, steps, dt=dt)
        X = inputs.node_positions(wl)
        ex = torch.tensor(np.sin(2 * np.pi * (X.sum(-1) - 1.5 * steps * dt)))[..., None]
        errs.append(float(l2(Q - ex, s)[0]))
    order = math.log(errs[0] / errs[2]) / math.log(9.0)
    assert order >= 4 - 0.3, (errs, order)
    assert errs[1] < 1e-6


# ------------------------------------------------------------- P10 Rusanov
def test_rusanov_is_upwind_for_advection():
    """P10: with s = |a|, the Rusanov flux is the exact upwind flux a q_upwind."""
    rng = np.random.default_rng(8)
    qL = torch.tensor(rng.standard_normal((6, 4, 1)))
    qR = torch.tensor(rng.standard_normal((6, 4, 1)))
    for a in (1.3, -0.7):
        lam = torch.full((6, 4), abs(a), dtype=torch.float64)
        F = ostep.rusanov(qL, qR, a * qL, a * qR, lam, lam)
        assert (F - (a * (qL if a > 0 else qR))).abs().max() < 1e-15


# ------------------------------------------- P11, P12 Euler bump (C2 physics)
def _bump(nc):
    wl = inputs.preset("C2").with_(n_cells=(nc,) * 3, length=1.0)
    s = ostep.Setup(wl.pde, 3, 4, wl.n_cells, wl.h, wl.pde_param)
    return wl, s, torch.tensor(inputs.initial_state(wl))


def test_c2_symmetry_and_steady_contact():
    """P11 / P12: the centred density bump with u = 0, p = 1 is a steady
    contact: after steps the momentum stays at round-off, energy is unchanged,
    only rho diffuses slightly; the state stays invariant under x <-> y
    permutation and x -> 1 - x reflection (cells and nodes)."""
    wl, s, Q = _bump(5)
    Q0 = Q.clone()
    for _ in range(2):
        dt = ostep.cfl_dt(ostep.max_wave_speed(Q, None, s), wl.cfl, s)
        Q = ostep.step(Q, None, dt, s)
    assert Q[..., 1:4].abs().max() < 1e-13
    assert (Q[..., 4] - Q0[..., 4]).abs().max() < 1e-13
    assert (Q[..., 0] - Q0[..., 0]).abs().max() < 1e-4      # O(h^(N+1)) diffusion, h = 0.2
    n = 5
    V = Q[..., 0].reshape(5, 5, 5, n, n, n)     # (cz, cy, cx, kz, ky, kx)
    assert (V - V.permute(0, 2, 1, 3, 5, 4)).abs().max() < 1e-14
    assert (V - V.flip(2).flip(5)).abs().max() < 1e-14


def test_translation_by_whole_cells():
    """P13: shifting the data by whole cells commutes with the step."""
    s, Q, _ = _rand_case(EULER, 3, 2, (4, 3, 2), 9)
    nx, ny, nz = s.n_cells
    def shift(X):
        return torch.roll(X.reshape(nz, ny, nx, -1, X.shape[-1]), (1, 2), dims=(2, 1)).reshape(X.shape)
    a = shift(ostep.step(Q, None, 0.01, s))
    b = ostep.step(shift(Q), None, 0.01, s)
    assert (a - b).abs().max() == 0.0


@pytest.mark.parametrize("pde", [EULER, ELASTIC])
def test_single_cell_axes_equal_tiled_grid(pde):
    """A grid with one cell along an axis (periodic neighbour = the cell
    itself) steps like the same data tiled twice along that axis."""
    s1, Q, par = _rand_case(pde, 3, 2, (1, 3, 1), 11)
    s2 = ostep.Setup(s1.pde_kind, 3, 2, (2, 3, 2), s1.h, s1.pde_param)
    def tile(X):
        Y = X.reshape(1, 3, 1, *X.shape[1:]).repeat(2, 1, 2, *([1] * (X.dim() - 1)))
        return Y.reshape(12, *X.shape[1:])
    a = ostep.step(Q, par, 0.01, s1)
    b = ostep.step(tile(Q), None if par is None else tile(par), 0.01, s2)
    assert (tile(a) - b).abs().max() <= 1e-15 * float(b.abs().max())


# ------------------------------------------ P14 step matrix and stability
def _step_matrix(s, dt, par=None):
    C, nn, m = s.ncells, s.n ** s.dim, s.m
    dim = C * nn * m
    S = np.zeros((dim, dim))
    for k in range(dim):
        e = torch.zeros(dim, dtype=torch.float64)
        e[k] = 1
        S[:, k] = ostep.step(e.view(C, nn, m), par, dt, s).reshape(-1).numpy()
    return S


def test_linear_step_matrix_conservation_and_consistency():
    """P14: the advection step matrix S is conservative (W^T S = W^T),
    preserves constants (S 1 = 1) and commutes with cell translations."""
    s = ostep.Setup(ADVECTION, 2, 2, (3, 3), 1 / 3, (1.0, 0.5))
    S = _step_matrix(s, 0.01)
    W = np.tile(node_weights(s).numpy(), s.ncells)
    assert np.abs(W @ S - W).max() < 1e-14
    assert np.abs(S @ np.ones(S.shape[0]) - 1).max() < 1e-14


def _symbol_blocks(s, dt):
    """Blocks S[c] = d(step cell c)/d(cell 0) of the linear step, from the step
    applied to every unit vector supported on cell 0 (3 cells per used axis:
    one step couples face neighbours only, so the offsets -1, 0, +1 do not
    alias), restricted to the nodes with k_j = 0 on the axes without
    transport (their data only ride along)."""
    C, nn, m = s.ncells, s.n ** s.dim, s.m
    cols = []
    for k in range(nn * m):
        e = torch.zeros(C * nn * m, dtype=torch.float64)
        e[k] = 1.0
        cols.append(ostep.step(e.view(C, nn, m), None, dt, s).reshape(C, nn * m))
    return torch.stack(cols, -1).numpy()


def _spectral_radius(s, dt, axes, nth):
    """max over the wavenumbers theta of the spectral radius of the
    amplification matrix G(theta) = sum_c S[c] exp(-i theta . offset(c))
    (von Neumann analysis of the periodic step; sampled on nth points per
    transported axis)."""
    B = _symbol_blocks(s, dt)
    n = s.n
    keep = [a for a in range(n ** s.dim)
            if all(((a // n ** i) % n) == 0 for i in range(s.dim) if i not in axes)]
    B = B[:, keep][:, :, keep]
    offs = []
    for c in range(s.ncells):
        o, r = [], c
        for i in range(s.dim):
            x = r % s.n_cells[i]
            r //= s.n_cells[i]
            o.append(x if x <= s.n_cells[i] // 2 else x - s.n_cells[i])
        offs.append(o)
    offs = np.array(offs, dtype=np.float64)
    th = np.linspace(0.0, 2 * np.pi, nth, endpoint=False)
    best = 0.0
    for t in itertools.product(*[th if i in axes else [0.0] for i in range(s.dim)]):
        G = np.tensordot(np.exp(-1j * (offs @ np.array(t))), B, axes=(0, 0))
        best = max(best, float(np.abs(np.linalg.eigvals(G)).max()))
    return best


def _rho_1d(N, C):
    s = ostep.Setup(ADVECTION, 2, N, (3, 1), 1 / 3, (1.0, 0.0))
    return _spectral_radius(s, C * s.h / (2 * N + 1), axes=(0,), nth=256)


@pytest.mark.parametrize("N", [3, 4, 7])
def test_time_step_stability_limit(N):
    """P14 (von Neumann): spectral radius rho of the periodic linear-advection
    step, dt = C h / ((2N+1) |a|).  The stated C = 0.9 is unstable for
    N >= 3 (rho = 1.55, 2.16, 5.55 for N = 3, 4, 7).  The limits C_N of the
    workload rule: N = 3 is exactly stable up to C_3 = 0.725 (rho <= 1 to
    round-off; the bisected limit is 0.7275); for N >= 4 the step has a
    weak growth at every C (rho - 1 ~ C^2: 4.3e-6 per step at the N = 4
    preset C = 0.9 C_4, 1.1e-4 at N = 7), and C_N marks where it jumps by
    orders of magnitude (rho >= 1.05 just above it)."""
    CN = inputs.STABLE_C[N]
    assert _rho_1d(N, 0.9) > 1.5
    if N == 3:
        assert _rho_1d(N, CN) <= 1 + 1e-12
        assert _rho_1d(N, 0.9 * CN) <= 1 + 1e-12
        assert _rho_1d(N, 1.015 * CN) > 1 + 1e-4
    else:
        weak = {4: 1e-5, 7: 2e-4}[N]
        r = _rho_1d(N, 0.9 * CN)
        assert 1.0 < r < 1 + weak
        assert _rho_1d(N, CN) < 1 + weak
        assert _rho_1d(N, 1.05 * CN) > 1.05
    if N == 4:   # growth of the weakest mode over the 100 steps of the Euler N = 4 workload
        assert _rho_1d(N, 0.9 * CN) ** 100 < 1 + 1e-3


def test_equal_speed_2d_stability():
    """P14 in 2D with equal speeds a = (1, 1) and the rule
    dt = C h / (d (2N+1) |a|_max): at N = 3 the stated C = 0.9 is unstable
    (rho = 1.61) and 0.9 C_3 is stable to round-off."""
    s = ostep.Setup(ADVECTION, 2, 3, (3, 3), 1 / 3, (1.0, 1.0))
    dt = lambda C: C * s.h / (2 * 7)
    assert _spectral_radius(s, dt(0.9), axes=(0, 1), nth=32) > 1.5
    assert _spectral_radius(s, dt(inputs.stable_cfl(3)), axes=(0, 1), nth=32) <= 1 + 1e-12


# --------------------------------------------------- flux / wave-speed pins
@pytest.mark.parametrize("kind,d", [(EULER, 3), (EULER, 2), (ACOUSTIC, 3), (ELASTIC, 3), (ELASTIC, 2)])
def test_wave_speed_is_largest_flux_jacobian_eigenvalue(kind, d):
    """The directional wave speed equals the largest |eigenvalue| of dF_i/dQ
    (autograd Jacobian + numpy eigvals); for Euler the eigenvalues are
    u_i - c, u_i (d times), u_i + c with c = sqrt(gamma p / rho)."""
    pde = make_pde(kind, d, (1.4,) if kind == EULER else ())
    rng = np.random.default_rng(10)
    m = pde.m
    if kind == EULER:
        q = torch.tensor([1.2, 0.3, -0.2, 0.1][:d + 1] + [3.1], dtype=torch.float64)
    else:
        q = torch.tensor(rng.standard_normal(m))
    par = torch.tensor([[1.1]] if kind == ACOUSTIC else [[1.3, 2.1, 0.9]], dtype=torch.float64)[0]
    for i in range(d):
        J = torch.autograd.functional.jacobian(lambda x: pde.flux(x, i, par), q).numpy()
        ev = np.linalg.eigvals(J)
        assert abs(np.abs(ev).max() - float(pde.speed(q[None], i, par[None]).max())) < 1e-12
        if kind == EULER:
            rho, ui = float(q[0]), float(q[1 + i] / q[0])
            p = float(pde.pressure(q))
            c = math.sqrt(1.4 * p / rho)
            assert np.allclose(sorted(ev.real), sorted([ui - c] + [ui] * d + [ui + c]), atol=1e-12)


def test_euler_flux_closed_form():
    """Sec. 7 Euler flux at a hand-computed state: rho=2, j=(1,0,0), E=5."""
    pde = make_pde(EULER, 3, (1.4,))
    q = torch.tensor([2.0, 1.0, 0.0, 0.0, 5.0])
    p = 0.4 * (5.0 - 0.5 * 1.0 / 2.0)          # 1.9
    F = pde.flux(q, 0, None).numpy()
    assert np.allclose(F, [1.0, 0.5 + p, 0.0, 0.0, 0.5 * (5.0 + p)], atol=1e-15)


# ------------------------------------------------ sampled step, diagnostics
def test_sampled_step_matches_full_step():
    s, Q, _ = _rand_case(EULER, 3, 2, (4, 3, 3), 11)
    full = ostep.step(Q, None, 0.01, s)
    cells = [0, 5, 17, 35]
    part = ostep.step_cells(Q, None, 0.01, s, cells)
    assert (full[cells] - part).abs().max() == 0.0


def test_point_values_interpolate_polynomials():
    wl = inputs.preset("C1").with_(n_cells=(3, 3))
    s = ostep.Setup(wl.pde, 2, 3, wl.n_cells, wl.h, wl.pde_param)
    X = inputs.node_positions(wl)
    Q = torch.tensor((X[..., 0] ** 3 - 2 * X[..., 1] ** 2 * X[..., 0]))[..., None]
    pts = np.array([[0.1, 0.77], [0.5, 0.2], [0.93, 0.41]])
    v = point_values(Q, s, pts).numpy()[:, 0]
    assert np.allclose(v, pts[:, 0] ** 3 - 2 * pts[:, 1] ** 2 * pts[:, 0], atol=1e-13)


# ------------------------------------------------------ P16 paper formulas
def test_corollary3_table_golden():
    """App. C table of Corollary 3 (paper, App. C "Proof for Corollary 3"):
    the relative footprint (2 + 6d) / ((d+1)(p+1) + 1 + 6d) to two decimals."""
    rows = []
    with open(os.path.join(GOLDEN, "corollary3_footprint.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                rows.append([float(x) for x in line.split()])
    assert len(rows) == 8
    for p, r2, r3 in rows:
        for d, r in ((2, r2), (3, r3)):
            val = (2 + 6 * d) / ((d + 1) * (p + 1) + 1 + 6 * d)
            assert abs(val - r) <= 0.005 + 1e-12, (p, d, val, r)
    assert (2 + 6 * 2) / (3 * 2 + 1 + 12) <= 0.875 + 1e-12   # the stated bound, p = 1


def test_corollary5_ratio_algebra():
    """Corollary 5: ((4d+2) C + 12d + 1) / (18d + 4) at C_rerun = 1 is
    (16d+3)/(18d+4): 0.875 for d = 2 and 0.879 for d = 3 (the printed 0.775
    does not follow from the formula)."""
    f = lambda d, C: ((4 * d + 2) * C + 12 * d + 1) / (18 * d + 4)
    assert abs(f(2, 1.0) - 0.875) < 1e-12
    assert abs(f(3, 1.0) - 51 / 58) < 1e-12
    assert abs(f(2, 2.0) - 1.125) < 1e-12
