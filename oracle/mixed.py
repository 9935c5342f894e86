"""The step with a reduced-precision predictor (precision emulation).

Oracle (test infrastructure only).  The paper computes in float64.  The mixed
form keeps the corrector (integrateVolume, Riemann, integrateFace, update,
Eq. (2) and Eq. (4)) in float64 and runs the space-time predictor of Eq. (3)
(Picard iteration, Sec. 3 "ADER-DG step 1") in a lower precision.  This module
rounds exactly the quantities that the mixed form rounds, so that the
reduced-precision GPU path can be compared with it element by element at a
tolerance set by float rounding (not by the precision gap to float64).

Precisions
----------
"fp64"  No rounding: the same steps in float64 (used to check that this
        module's arrangement of the step equals the plain one).
"fp32"  The Picard iteration in float32: q, the fluxes F_i(q), the spatial
        contractions with D and the time contraction with P.
"bf16"  As "fp32", except that each spatial contraction takes bfloat16
        inputs with float32 accumulation: the flux differences F - F_ref
        (below) are rounded to bfloat16 (round to nearest, ties to even) and
        D is carried as the sum D_hi + D_lo of two bfloat16 numbers
        (D_hi = bf16(fl32(D)), D_lo = bf16(fl32(D - D_hi))), a 16-bit
        operator that float32 holds exactly.

Contraction against a reference flux (both precisions): the rows of D sum to
zero (the derivative of a constant vanishes), so D F = D (F - F_ref 1) for
any F_ref constant along the contracted axis.  With F_ref a flux of the same
pencil a constant flux has exactly zero derivative in any precision, and the
rounded inputs carry errors relative to the variation along the pencil, not
to the flux itself.  F_ref is the flux at the first node for n < 5, at the
middle node for odd n >= 5 and the mean of the middle pair for even n >= 6.

What stays float64: the time averages of q and F_i (accumulated in float64
from the float32 values), the volume term, the extrapolation to the faces
(whose results are then stored in float32: the hull), the Rusanov solve, the
face lift and the update.  For the linear PDEs the time-averaged flux is
taken as F_i(qbar) in float64 (equal to the average of F_i(q) since F_i is
linear), the hull keeps only the q traces, and the face fluxes are rebuilt
from them in float64; so a constant state stays exactly constant here too.
"""

import numpy as np
import torch

from . import step as ostep

F64 = torch.float64
F32 = torch.float32


def bf16_rne(x):
    """Round float32 values to bfloat16 (nearest, ties to even), as float32."""
    return x.to(torch.bfloat16).to(F32)


def operator_bf16_pair(D):
    """(D_hi, D_lo) as float32 tensors holding bfloat16 values:
    D_hi = bf16(fl32(D)), D_lo = bf16(fl32(D - D_hi)) (D in float64)."""
    D = torch.as_tensor(np.asarray(D), dtype=F64)
    hi = bf16_rne(D.to(F32))
    lo = bf16_rne((D - hi.to(F64)).to(F32))
    return hi, lo


def reference_flux(F, dim, n):
    """F_ref along tensor dimension dim (kept as a size-1 dimension)."""
    if n < 5:
        return F.narrow(dim, 0, 1)
    if n % 2 == 1:
        return F.narrow(dim, n // 2, 1)
    return 0.5 * (F.narrow(dim, n // 2 - 1, 1) + F.narrow(dim, n // 2, 1))


def _contract(x, M, dim):
    """out[.., a, ..] = sum_j M[a][j] x[.., j, ..] along dim, in x's dtype."""
    y = torch.movedim(x, dim, -1) @ M.T.to(x.dtype)
    return torch.movedim(y, -1, dim)


def predictor_mixed(u, par, dt, s, precision):
    """The space-time predictor of Eq. (3) with R Picard iterations in the
    reduced precision: q <- fl32(u) - fl32(dt/h) P (sum_i D_i (F_i(q) - F_ref,i)),
    starting from q = fl32(u) on every time node.

    u: (C, n, .., n, m) float64; returns q (C, n_t, n, .., n, m) in the
    working precision (float32; float64 for "fp64")."""
    C, d, n = u.shape[0], s.dim, s.n
    parq = ostep._par_view(par, d + 1, C)
    wt = F64 if precision == "fp64" else F32
    u32 = u.to(wt)
    parq = None if parq is None else parq.to(wt)
    P = torch.as_tensor(s.tab.P, dtype=F64).to(wt)
    if precision in ("fp32", "fp64"):
        Dop = torch.as_tensor(s.tab.D, dtype=F64).to(wt)
        rnd = lambda x: x
    elif precision == "bf16":
        hi, lo = operator_bf16_pair(s.tab.D)
        Dop = hi + lo                     # exact in float32
        rnd = bf16_rne
    else:
        raise ValueError(precision)
    c = torch.tensor(dt / s.h, dtype=F64).to(wt)
    q = u32.unsqueeze(1).expand(C, n, *u32.shape[1:]).clone()
    for _ in range(s.R):
        rhs = None
        for i in range(d):
            dim = -(i + 2)
            Fi = s.pde.flux(q, i, parq)
            X = rnd(Fi - reference_flux(Fi, dim, n))
            t = _contract(X, Dop, dim)
            rhs = t if rhs is None else rhs + t
        q = u32.unsqueeze(1) - c * _contract(rhs, P, 1)
    return q


def step_mixed(Q, par, dt, s, precision):
    """Q(T + dt) from Q(T) with the predictor in ``precision`` and everything
    after it in float64 (Eq. (2), (4), (6)); the hull is stored in the
    predictor's working precision.
    Q: (C, n^d, m) float64."""
    C = Q.shape[0]
    u = ostep._spatial(Q, s)
    q = predictor_mixed(u, par, dt, s, precision)
    parq = ostep._par_view(par, s.dim + 1, C)
    parw = None if parq is None else parq.to(q.dtype)
    w = torch.as_tensor(s.tab.w, dtype=F64)
    qbar = ostep.project(q.to(F64), w, dim=1)
    if s.pde.linear:
        Fbar = [s.pde.flux(qbar, i, ostep._par_view(par, s.dim, C)) for i in range(s.dim)]
    else:
        Fbar = [ostep.project(s.pde.flux(q, i, parw).to(F64), w, dim=1) for i in range(s.dim)]
    Qt = ostep.integrate_volume(u, Fbar, dt, s)
    hull = q.dtype       # the hull is stored in the predictor's precision
    tr = [tuple(x.to(hull).to(F64) for x in t) for t in ostep.extrapolate(qbar, Fbar, s)]
    if s.pde.linear:
        # linear PDEs keep only the q traces; the face fluxes are rebuilt from
        # them in float64 with the owning cell's material
        pf = ostep._par_view(par, s.dim - 1, C)
        tr = [(qL, qR, s.pde.flux(qL, i, pf), s.pde.flux(qR, i, pf))
              for i, (qL, qR, _, _) in enumerate(tr)]
    plus, minus = ostep.neighbor_index(s.n_cells)
    Fp, Fm = [], []
    for i in range(s.dim):
        pi = torch.as_tensor(plus[i])
        mi = torch.as_tensor(minus[i])
        tr_plus = tuple(t[pi] for t in tr[i])
        par_plus = None if par is None else par[pi]
        F = ostep.face_fluxes(tr[i], tr_plus, par, par_plus, i, s)
        Fp.append(F)
        Fm.append(F[mi])
    Qn = ostep.integrate_face(Qt, Fp, Fm, dt, s)
    return Qn.reshape(C, -1, s.m)


def run_mixed(Q, par, s, steps, precision, dts):
    """Steps with the given time steps (the float64 run's sequence)."""
    for k in range(steps):
        Q = step_mixed(Q, par, float(dts[k]), s, precision)
    return Q
