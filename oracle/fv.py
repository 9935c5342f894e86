"""Finite-volume subcell patches: the limiter's subgrid and its step.

Oracle (test infrastructure only).  Sec. 3 ("Finite Volume limiter") gives a
troubled ADER-DG cell of order p a regular Cartesian subgrid of (2p+1)^d
finite-volume cells, advanced by a finite-volume scheme and projected back
onto the DG space by averaging.  App. A, Corollary 8, casts first-order
finite volumes with Rusanov fluxes into the predictor-corrector formalism:
p = 0, the predictor is the identity, the traces of a cell are its own value
and flux, so one step is
    Q(T + dT) = (id + dT computeRusanovFluxes o id_{c -> dc}) Q(T).

Here every cell carries a patch (the subgrid of the whole domain):

* ``P[cell][subcell][var]``: the S^d subcell averages of a cell (S = 2N + 1),
  subcells lexicographic with the x index fastest, like the nodes of Q;
* ``project``: DG nodal values -> subcell averages, the exact average of the
  cell's polynomial over each subcell (a Gauss rule with n points per
  subcell, exact for degree N);
* ``reconstruct``: subcell averages -> DG nodal values, the least-squares
  inverse of ``project`` per axis, R = (Pi^T Pi)^-1 Pi^T (exact for data that
  came from a polynomial of degree N, since S >= n);
* ``fv_step``: one first-order Rusanov step on the subgrid with spacing
  h / S, written directly as the textbook scheme on the fine grid (periodic
  shifts of the fine-grid array): F*_{i+1/2} = (f_L + f_R)/2 -
  s (Q_R - Q_L)/2 with s = max(lambda_L, lambda_R) per face, and
  Q <- Q - dt S / h (F*_{i+1/2} - F*_{i-1/2}) summed over the axes.  A
  subcell's material parameters are those of its cell (per-cell constants in
  conservative flux form, as for the DG step).
"""

import numpy as np
import torch

from .tables import barycentric_weights, gauss_legendre_unit, lagrange_values

F64 = torch.float64


def subcells(order):
    """S = 2N + 1 subcells per axis (the subgrid resolution of Sec. 3)."""
    return 2 * order + 1


def average_matrix(order):
    """Pi[s][j] = average over subcell s of phi_j = S int_{s/S}^{(s+1)/S} phi_j,
    by an n-point Gauss rule on each subcell (exact for phi_j of degree N)."""
    n, S = order + 1, subcells(order)
    xi, _ = gauss_legendre_unit(n)
    lam = barycentric_weights(xi)
    zq, wq = gauss_legendre_unit(n)
    Pi = np.zeros((S, n))
    for s_ in range(S):
        for q in range(n):
            Pi[s_] += wq[q] * lagrange_values(xi, lam, (s_ + zq[q]) / S)
    return Pi


def reconstruct_matrix(order):
    """R = (Pi^T Pi)^-1 Pi^T: least squares from S subcell averages to n nodes."""
    Pi = average_matrix(order)
    return np.linalg.solve(Pi.T @ Pi, Pi.T)


def _apply_axes(X, M, d, npts_in, m):
    """Contract each of the d spatial axes of X (C, npts_in^d, m) with M
    (out x in); spatial axis i is tensor dimension -(i + 2)."""
    C = X.shape[0]
    T = X.reshape(C, *([npts_in] * d), m)
    Mt = torch.as_tensor(M, dtype=F64)
    for i in range(d):
        dim = T.dim() - (i + 2)
        T = torch.movedim(torch.movedim(T, dim, -1) @ Mt.T, -1, dim)
    return T.reshape(C, -1, m)


def project(Q, s):
    """Subcell averages P (C, S^d, m) of the DG solution Q (C, n^d, m)."""
    return _apply_axes(Q, average_matrix(s.order), s.dim, s.n, s.m)


def reconstruct(P, s):
    """DG nodal values (C, n^d, m) from subcell averages P (C, S^d, m)."""
    return _apply_axes(P, reconstruct_matrix(s.order), s.dim, subcells(s.order), s.m)


def to_fine(X, s):
    """Patch layout (C, S^d, k) -> fine grid (n_z S, n_y S, n_x S, k), the
    fine x index fastest (fine index along axis i = cell_i S + subcell_i)."""
    d, S = s.dim, subcells(s.order)
    nc = list(reversed(s.n_cells))                        # (.., ny, nx)
    k = X.shape[-1]
    T = X.reshape(*nc, *([S] * d), k)                      # cell axes, then subcell axes
    perm = []
    for a in range(d):                                     # interleave (cell_a, sub_a)
        perm += [a, d + a]
    T = T.permute(*perm, 2 * d)
    return T.reshape(*[nc[a] * S for a in range(d)], k)


def from_fine(G, s):
    """Inverse of ``to_fine``."""
    d, S = s.dim, subcells(s.order)
    nc = list(reversed(s.n_cells))
    k = G.shape[-1]
    shape = []
    for a in range(d):
        shape += [nc[a], S]
    T = G.reshape(*shape, k)
    perm = [2 * a for a in range(d)] + [2 * a + 1 for a in range(d)]
    T = T.permute(*perm, 2 * d)
    return T.reshape(int(np.prod(nc)), S ** d, k)


def fv_step(P, par, dt, s):
    """One first-order Rusanov finite-volume step on the subgrid (App. A,
    Corollary 8), periodic, subcell width h / S.  P: (C, S^d, m)."""
    d, S = s.dim, subcells(s.order)
    G = to_fine(P, s)                                      # (.., x, m), axis i at dim d-1-i
    Gp = None if par is None else to_fine(
        par.reshape(par.shape[0], 1, par.shape[-1]).expand(par.shape[0], S ** d, par.shape[-1]), s)
    hs = s.h / S
    out = G.clone()
    for i in range(d):
        ax = d - 1 - i
        GR = torch.roll(G, -1, dims=ax)                    # right neighbour along +e_i
        pL = Gp
        pR = None if Gp is None else torch.roll(Gp, -1, dims=ax)
        fL = s.pde.flux(G, i, pL)
        fR = s.pde.flux(GR, i, pR)
        sv = torch.maximum(s.pde.speed(G, i, pL), s.pde.speed(GR, i, pR)).unsqueeze(-1)
        Fh = 0.5 * (fL + fR) - 0.5 * sv * (GR - G)         # flux on the face i + 1/2
        out = out - (dt / hs) * (Fh - torch.roll(Fh, 1, dims=ax))
    return from_fine(out, s)
