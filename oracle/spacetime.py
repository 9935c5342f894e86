"""The step with space-time traces (Table 1's cardinalities), FP64.

Oracle (test infrastructure only).  ``extrapolate`` keeps Q* and F_i(Q*) on
the 2d faces at every time node (4 d m n^d values per cell, Table 1 task
extrapolate), ``solveRiemann`` solves the Rusanov problem at every time node
of every face node with one s per face and time node (the maximum over the
face nodes and both sides of the directional speed at that time node), and
integrateFace uses the time integral sum_t w_t F*(t).  The volume term and
the update are those of ``step.step``.  With a constant wave speed (linear
advection) this is the time-integrated step exactly.

``step_st_mixed`` is the same step with the predictor in a reduced precision
(``mixed.predictor_mixed``): it rounds what ``mixed.step_mixed`` rounds, and
the hull it stores between extrapolate and solveRiemann holds every time
node's traces in the predictor's precision.
"""

import torch

from . import mixed
from . import step as ostep

F64 = torch.float64


def extrapolate_st(q, par, s):
    """Traces at every time node: for axis i (qL, qR, fL, fR), each of shape
    (C, n_t, face dims.., m): q and F_i(q) at xi_i = 0 (L) and 1 (R)."""
    C, d = q.shape[0], s.dim
    parq = ostep._par_view(par, d + 1, C)
    out = []
    for i in range(d):
        dim = -(i + 2)
        Fi = s.pde.flux(q, i, parq)
        out.append((ostep.project(q, s.tab.FL, dim), ostep.project(q, s.tab.FR, dim),
                    ostep.project(Fi, s.tab.FL, dim), ostep.project(Fi, s.tab.FR, dim)))
    return out


def face_fluxes_st(tr_self, tr_plus, par_self, par_plus, i, s):
    """Time integral of the Rusanov flux of each time node on the face between
    a cell (left) and its +e_i neighbour: sum_t w_t F*(t), with
    F*(t) = (fL + fR)/2 - s(t) (qR - qL)/2 and s(t) the maximum over the face
    nodes and both sides at time node t."""
    qL, fL = tr_self[1], tr_self[3]
    qR, fR = tr_plus[0], tr_plus[2]
    C = qL.shape[0]
    pL = ostep._par_view(par_self, s.dim, C)
    pR = ostep._par_view(par_plus, s.dim, C)
    lam = torch.maximum(s.pde.speed(qL, i, pL), s.pde.speed(qR, i, pR))   # (C, n_t, face..)
    smax = lam.reshape(C, s.n, -1).max(dim=2).values                       # (C, n_t)
    sv = smax.reshape(C, s.n, *([1] * (qL.dim() - 2)))
    F = 0.5 * (fL + fR) - 0.5 * sv * (qR - qL)
    return ostep.project(F, s.tab.w, dim=1)


def step_st(Q, par, dt, s):
    """Q(T + dt) from Q(T) with space-time traces and per-time-node Rusanov."""
    C = Q.shape[0]
    u = ostep._spatial(Q, s)
    q = ostep.predictor(u, par, dt, s)
    _, Fbar = ostep.time_average(q, par, s)
    Qt = ostep.integrate_volume(u, Fbar, dt, s)
    tr = extrapolate_st(q, par, s)
    plus, minus = ostep.neighbor_index(s.n_cells)
    Fp, Fm = [], []
    for i in range(s.dim):
        pi = torch.as_tensor(plus[i])
        mi = torch.as_tensor(minus[i])
        tr_plus = tuple(t[pi] for t in tr[i])
        par_plus = None if par is None else par[pi]
        F = face_fluxes_st(tr[i], tr_plus, par, par_plus, i, s)
        Fp.append(F)
        Fm.append(F[mi])
    return ostep.integrate_face(Qt, Fp, Fm, dt, s).reshape(C, -1, s.m)


def step_st_mixed(Q, par, dt, s, precision):
    """Q(T + dt) with space-time traces and the predictor of Eq. (3) in
    ``precision`` ("fp64", "fp32", "bf16"; see ``mixed``).

    The Picard iterate q at every space-time node comes in the working
    precision.  Its time averages (float64 sums of the rounded values; for
    the linear PDEs Fbar_i = F_i(qbar) in float64), the volume term, the
    extrapolation of q(t) and F_i(q(t)) to the faces at every time node (the
    fluxes evaluated in the working precision, the projection in float64),
    the per-time-node Rusanov solves, the face lift and the update are
    float64; the face values are rounded to the working precision once, when
    stored in the hull.  The linear PDEs store only the q traces and rebuild
    the face fluxes from them in float64 with the owning cell's material."""
    C, d = Q.shape[0], s.dim
    u = ostep._spatial(Q, s)
    q = mixed.predictor_mixed(u, par, dt, s, precision)
    hull = q.dtype
    parq = ostep._par_view(par, d + 1, C)
    parw = None if parq is None else parq.to(hull)
    w = torch.as_tensor(s.tab.w, dtype=F64)
    q64 = q.to(F64)
    qbar = ostep.project(q64, w, dim=1)
    if s.pde.linear:
        Fbar = [s.pde.flux(qbar, i, ostep._par_view(par, d, C)) for i in range(d)]
    else:
        Fbar = [ostep.project(s.pde.flux(q, i, parw).to(F64), w, dim=1) for i in range(d)]
    Qt = ostep.integrate_volume(u, Fbar, dt, s)
    stored = lambda x: x.to(hull).to(F64)
    pf = ostep._par_view(par, d, C)       # over (C, n_t, face nodes.., m)
    tr = []
    for i in range(d):
        dim = -(i + 2)
        qL = stored(ostep.project(q64, s.tab.FL, dim))
        qR = stored(ostep.project(q64, s.tab.FR, dim))
        if s.pde.linear:
            fL, fR = s.pde.flux(qL, i, pf), s.pde.flux(qR, i, pf)
        else:
            Fi = s.pde.flux(q, i, parw).to(F64)
            fL = stored(ostep.project(Fi, s.tab.FL, dim))
            fR = stored(ostep.project(Fi, s.tab.FR, dim))
        tr.append((qL, qR, fL, fR))
    plus, minus = ostep.neighbor_index(s.n_cells)
    Fp, Fm = [], []
    for i in range(d):
        pi = torch.as_tensor(plus[i])
        mi = torch.as_tensor(minus[i])
        tr_plus = tuple(t[pi] for t in tr[i])
        par_plus = None if par is None else par[pi]
        F = face_fluxes_st(tr[i], tr_plus, par, par_plus, i, s)
        Fp.append(F)
        Fm.append(F[mi])
    return ostep.integrate_face(Qt, Fp, Fm, dt, s).reshape(C, -1, s.m)
