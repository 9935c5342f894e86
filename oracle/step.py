"""One explicit ADER-DG step on a uniform periodic Cartesian grid, in FP64.

Oracle (test infrastructure only).  Each function names the passage of the
paper it follows.  Data layout (shared with the GPU path only as a convention):

* ``Q[cell][node][var]``: cells lexicographic with x fastest
  (c = ix + nx (iy + ny iz)); nodes lexicographic with k_x fastest; the m
  variables innermost.
* Face traces of axis i: the n^(d-1) face nodes ordered with the lower axes
  fastest (the spatial index with coordinate i removed).

Internally a cell's spatial tensor is viewed as (..., k_{d-1}, ..., k_0, m),
so spatial axis i sits at tensor dimension ``-(i + 2)``.
"""

from dataclasses import dataclass

import numpy as np
import torch

from .pde import make_pde
from .tables import make_tables

F64 = torch.float64


@dataclass
class Setup:
    """Grid and method parameters of one run (plain numbers, no arrays)."""
    pde_kind: int
    dim: int
    order: int
    n_cells: tuple          # (nx, ny[, nz])
    h: float                # uniform cell width
    pde_param: tuple = ()
    picard_iters: int = 0   # 0 -> N + 1 (reading of the unstated count)

    def __post_init__(self):
        self.n_cells = tuple(int(x) for x in self.n_cells)
        assert len(self.n_cells) == self.dim
        self.tab = make_tables(self.order)
        self.pde = make_pde(self.pde_kind, self.dim, self.pde_param)

    @property
    def n(self):
        return self.order + 1

    @property
    def m(self):
        return self.pde.m

    @property
    def ncells(self):
        return int(np.prod(self.n_cells))

    @property
    def R(self):
        return self.picard_iters if self.picard_iters > 0 else self.order + 1


def _t(a):
    return torch.as_tensor(np.asarray(a), dtype=F64)


def contract(x, M, dim):
    """out[.., a, ..] = sum_j M[a][j] x[.., j, ..] along tensor dimension dim."""
    y = torch.movedim(x, dim, -1) @ _t(M).T
    return torch.movedim(y, -1, dim)


def project(x, v, dim):
    """sum_j v[j] x[.., j, ..], removing tensor dimension dim."""
    return torch.tensordot(torch.movedim(x, dim, -1), _t(v), dims=([x.dim() - 1], [0]))


def _spatial(Q, s):
    C = Q.shape[0]
    return Q.reshape(C, *([s.n] * s.dim), s.m)


def _par_view(par, ndim_between, C):
    if par is None:
        return None
    return par.reshape(C, *([1] * ndim_between), par.shape[-1])


# ---------------------------------------------------------------------------
# ADER-DG step 1: space-time predictor (Eq. (3), Picard, Sec. 3)
# ---------------------------------------------------------------------------
def predictor(u, par, dt, s, iters=None, tol=None, max_iters=200):
    """Space-time predictor of every cell: q at the n^(d+1) space-time nodes.

    Eq. (3) restricted to one cell, tested with theta_k(tau) phi_a(x) and
    integrated by parts in time with the cell state u as upwind value at
    tau = 0, with F(q) collocated at the nodes (quadrature-free):
        K1 q = FL u - dt diag(w) rhs,  rhs = sum_i (1/h) D_i F_i(q),
    solved by the Picard iteration q <- u - dt P rhs(q) from q = u.
    ``iters`` fixes the count (default N + 1); ``tol`` instead iterates until
    the update is below tol * max|q| (used by the brute-force pins).

    u: (C, n, .., n, m) spatial tensor; returns (C, n_t, n, .., n, m).
    """
    C, d, n = u.shape[0], s.dim, s.n
    parq = _par_view(par, d + 1, C)
    q = u.unsqueeze(1).expand(C, n, *u.shape[1:]).clone()
    R = s.R if iters is None else iters
    if tol is not None:
        R = max_iters
    for r in range(R):
        rhs = None
        for i in range(d):
            Fi = s.pde.flux(q, i, parq)
            t = contract(Fi, s.tab.D, dim=-(i + 2))
            rhs = t if rhs is None else rhs + t
        q_new = u.unsqueeze(1) - (dt / s.h) * contract(rhs, s.tab.P, dim=1)
        if tol is not None:
            delta = (q_new - q).abs().max()
            q = q_new
            if delta <= tol * q.abs().max():
                break
        else:
            q = q_new
    return q


def time_average(q, par, s):
    """qbar = sum_l w_l q_l and Fbar_i = sum_l w_l F_i(q_l) (1/dt times the
    time integral over the step)."""
    C, d = q.shape[0], s.dim
    parq = _par_view(par, d + 1, C)
    qbar = project(q, s.tab.w, dim=1)
    Fbar = [project(s.pde.flux(q, i, parq), s.tab.w, dim=1) for i in range(d)]
    return qbar, Fbar


def integrate_volume(u, Fbar, dt, s):
    """integrateVolume, brought forward behind predict (Technique 1):
    Q~ = u + dt V, V_a = (1/h) sum_i sum_j Kv[a_i][j] Fbar_i[a | a_i <- j]
    (Eq. (2) first term, divided by the diagonal GL mass matrix)."""
    V = None
    for i in range(s.dim):
        t = contract(Fbar[i], s.tab.Kv, dim=-(i + 2))
        V = t if V is None else V + t
    return u + (dt / s.h) * V


def extrapolate(qbar, Fbar, s):
    """extrapolate (Table 1): time-integrated traces on the 2d faces.

    For axis i returns (qL, qR, fL, fR): qbar and Fbar_i (flux along +e_i)
    evaluated at xi_i = 0 (L) and xi_i = 1 (R); each (C, n^(d-1) face dims, m).
    """
    out = []
    for i in range(s.dim):
        dim = -(i + 2)
        out.append((project(qbar, s.tab.FL, dim), project(qbar, s.tab.FR, dim),
                    project(Fbar[i], s.tab.FL, dim), project(Fbar[i], s.tab.FR, dim)))
    return out


# ---------------------------------------------------------------------------
# ADER-DG step 2 and 3: Rusanov (Eq. (4)) and the corrector (Eq. (2))
# ---------------------------------------------------------------------------
def rusanov(qL, qR, fL, fR, lamL, lamR):
    """Rusanov / local Lax-Friedrichs flux along +e_i on one face.

    s = max over the face nodes and both sides of the directional wave speed;
    F* = (fL + fR)/2 - s (qR - qL)/2.  qL.. have shape (F, face dims.., m),
    lamL/lamR (F, face dims..)."""
    smax = torch.maximum(lamL, lamR).reshape(lamL.shape[0], -1).max(dim=1).values
    sv = smax.reshape(-1, *([1] * (qL.dim() - 1)))
    return 0.5 * (fL + fR) - 0.5 * sv * (qR - qL)


def neighbor_index(n_cells):
    """plus[i][c] = index of c + e_i, minus[i][c] = index of c - e_i (periodic)."""
    d = len(n_cells)
    grid = np.arange(int(np.prod(n_cells))).reshape(tuple(reversed(n_cells)))
    plus, minus = [], []
    for i in range(d):
        ax = d - 1 - i
        plus.append(np.roll(grid, -1, axis=ax).reshape(-1))
        minus.append(np.roll(grid, 1, axis=ax).reshape(-1))
    return plus, minus


def face_fluxes(tr_self, tr_plus, par_self, par_plus, i, s):
    """Rusanov flux on the face between a cell (left) and its +e_i neighbour.

    tr_*: the (qL, qR, fL, fR) traces of axis i of the two cells."""
    qL, fL = tr_self[1], tr_self[3]        # right-face trace of the left cell
    qR, fR = tr_plus[0], tr_plus[2]        # left-face trace of the right cell
    C = qL.shape[0]
    pL = _par_view(par_self, s.dim - 1, C)
    pR = _par_view(par_plus, s.dim - 1, C)
    lamL = s.pde.speed(qL, i, pL)
    lamR = s.pde.speed(qR, i, pR)
    return rusanov(qL, qR, fL, fR, lamL, lamR)


def integrate_face(Qt, Fplus, Fminus, dt, s):
    """integrateFace + update:
    Q_a = Q~_a - (dt/h) sum_i (LR[a_i] F*_{i,+}[a_!i] - LL[a_i] F*_{i,-}[a_!i]),
    with F* along +e_i on the cell's right (+) and left (-) face of axis i
    (Eq. (2) second term divided by the GL mass matrix)."""
    Qn = Qt
    n = s.n
    for i in range(s.dim):
        dim = Qt.dim() - (i + 2)
        shape = [1] * Qt.dim()
        shape[dim] = n
        LR = _t(s.tab.LR).reshape(shape)
        LL = _t(s.tab.LL).reshape(shape)
        Qn = Qn - (dt / s.h) * (LR * Fplus[i].unsqueeze(dim) - LL * Fminus[i].unsqueeze(dim))
    return Qn


def step(Q, par, dt, s, iters=None):
    """Q(T + dt) from Q(T): Eq. (6), predict evaluated once per cell.

    Q: (C, n^d, m) float64; par: (C, npar) or None; dt: python float.
    """
    C = Q.shape[0]
    u = _spatial(Q, s)
    q = predictor(u, par, dt, s, iters=iters)
    qbar, Fbar = time_average(q, par, s)
    Qt = integrate_volume(u, Fbar, dt, s)
    tr = extrapolate(qbar, Fbar, s)
    plus, minus = neighbor_index(s.n_cells)
    Fp, Fm = [], []
    for i in range(s.dim):
        pi = torch.as_tensor(plus[i])
        mi = torch.as_tensor(minus[i])
        tr_plus = tuple(t[pi] for t in tr[i])
        par_plus = None if par is None else par[pi]
        F = face_fluxes(tr[i], tr_plus, par, par_plus, i, s)
        Fp.append(F)
        Fm.append(F[mi])
    Qn = integrate_face(Qt, Fp, Fm, dt, s)
    return Qn.reshape(C, -1, s.m)


def step_cells(Q, par, dt, s, cells, iters=None):
    """Q(T + dt) at the listed cells only (for sampled parity at full size).

    Runs the predictor on the listed cells and their 2d face neighbours and
    the corrector on the listed cells; the arithmetic is that of ``step``.
    """
    cells = np.asarray(cells, dtype=np.int64)
    plus, minus = neighbor_index(s.n_cells)
    need = np.unique(np.concatenate([cells] + [p[cells] for p in plus] +
                                    [m[cells] for m in minus]))
    pos = {int(c): k for k, c in enumerate(need)}
    Qs = Q[torch.as_tensor(need)]
    ps = None if par is None else par[torch.as_tensor(need)]
    u = _spatial(Qs, s)
    q = predictor(u, ps, dt, s, iters=iters)
    qbar, Fbar = time_average(q, ps, s)
    Qt = integrate_volume(u, Fbar, dt, s)
    tr = extrapolate(qbar, Fbar, s)
    sel = torch.as_tensor([pos[int(c)] for c in cells])
    Fp, Fm = [], []
    for i in range(s.dim):
        ip = torch.as_tensor([pos[int(plus[i][c])] for c in cells])
        im = torch.as_tensor([pos[int(minus[i][c])] for c in cells])
        t_self = tuple(t[sel] for t in tr[i])
        t_plus = tuple(t[ip] for t in tr[i])
        t_minus = tuple(t[im] for t in tr[i])
        p_self = None if ps is None else ps[sel]
        p_plus = None if ps is None else ps[ip]
        p_minus = None if ps is None else ps[im]
        Fp.append(face_fluxes(t_self, t_plus, p_self, p_plus, i, s))
        Fm.append(face_fluxes(t_minus, t_self, p_minus, p_self, i, s))
    Qn = integrate_face(Qt[sel], Fp, Fm, dt, s)
    return Qn.reshape(len(cells), -1, s.m)


# ---------------------------------------------------------------------------
# calcTimeStep (Sec. 3 "Time stepping"; Alg. 1)
# ---------------------------------------------------------------------------
def max_wave_speed(Q, par, s):
    """max over cells, nodes and axes of the directional wave speed."""
    C = Q.shape[0]
    pv = None if par is None else par.reshape(C, 1, par.shape[-1])
    return max(float(s.pde.speed(Q, i, pv).max()) for i in range(s.dim))


def cfl_dt(lam, cfl, s):
    """dt = C h / (d (2N + 1) lambda_max)."""
    return cfl * s.h / (s.dim * (2 * s.order + 1) * lam)


def run(Q, par, s, steps, cfl=None, dt=None):
    """Alg. 1 (standard time stepping): fixed dt, or dt recomputed from the
    state at the start of every step when ``cfl`` is given.
    Returns (Q, list of dts)."""
    dts = []
    for _ in range(steps):
        dtn = dt if cfl is None else cfl_dt(max_wave_speed(Q, par, s), cfl, s)
        Q = step(Q, par, dtn, s)
        dts.append(dtn)
    return Q, dts
