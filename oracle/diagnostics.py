"""Diagnostics on a nodal DG state (oracle, test infrastructure only).

GL quadrature on each cell: int_cell f dx ~= h^d sum_a W_a f_a with the
tensor-product weights W_a = prod_i w_{a_i} (Sec. 3 basis; exact for the
polynomial degrees met here).
"""

import numpy as np
import torch

from .tables import barycentric_weights, lagrange_values

F64 = torch.float64


def node_weights(s):
    """W_a for a = lexicographic node index with k_x fastest."""
    w = s.tab.w
    W = np.ones(1)
    for _ in range(s.dim):
        W = np.kron(w, W)          # new (higher) axis varies slowest
    return torch.as_tensor(W, dtype=F64)


def totals(Q, s):
    """Conserved totals M_v = sum_c h^d sum_a W_a Q[c][a][v]."""
    W = node_weights(s)
    return (s.h ** s.dim) * torch.einsum("a,cav->v", W, Q)


def l2(Q, s):
    """Per-variable L2 norm over the domain."""
    W = node_weights(s)
    return torch.sqrt((s.h ** s.dim) * torch.einsum("a,cav->v", W, Q * Q))


def rel_l2(Q, ref, s, floor=1e-8):
    """Per-variable relative L2 error; absolute where the reference norm is
    below floor * (largest variable norm)."""
    e = l2(Q - ref, s)
    r = l2(ref, s)
    big = float(r.max())
    out = torch.where(r < floor * big, e, e / torch.where(r > 0, r, torch.ones_like(r)))
    return out


def point_values(Q, s, points):
    """Evaluate the DG polynomial of variable set Q at physical points
    (periodic domain [0, nx h) x ...): sum_a Q[c(x)][a] prod_i phi_{a_i}(xi_i)."""
    lam = barycentric_weights(s.tab.xi)
    pts = np.asarray(points, dtype=np.float64)
    out = []
    for x in pts:
        idx, basis = [], None
        for i in range(s.dim):
            L = s.n_cells[i] * s.h
            xi_ = (x[i] % L) / s.h
            ci = min(int(np.floor(xi_)), s.n_cells[i] - 1)
            idx.append(ci)
            phi = lagrange_values(s.tab.xi, lam, xi_ - ci)
            basis = phi if basis is None else np.kron(phi, basis)
        c = 0
        for i in reversed(range(s.dim)):
            c = c * s.n_cells[i] + idx[i]
        out.append(torch.as_tensor(basis, dtype=F64) @ Q[c])
    return torch.stack(out)


def basis_rows(s, points):
    """(cell index, basis row) per point so that value = row @ Q[cell]; used to
    build differentiable receiver sampling."""
    lam = barycentric_weights(s.tab.xi)
    cells, rows = [], []
    for x in np.asarray(points, dtype=np.float64):
        idx, basis = [], None
        for i in range(s.dim):
            L = s.n_cells[i] * s.h
            xi_ = (x[i] % L) / s.h
            ci = min(int(np.floor(xi_)), s.n_cells[i] - 1)
            idx.append(ci)
            phi = lagrange_values(s.tab.xi, lam, xi_ - ci)
            basis = phi if basis is None else np.kron(phi, basis)
        c = 0
        for i in reversed(range(s.dim)):
            c = c * s.n_cells[i] + idx[i]
        cells.append(c)
        rows.append(basis)
    return np.array(cells), torch.as_tensor(np.array(rows), dtype=F64)


def kinetic_energy(Q, s):
    """KE = sum_c h^d sum_a W_a |j|^2 / (2 rho) (Euler)."""
    W = node_weights(s)
    rho = Q[..., 0]
    j = Q[..., 1:1 + s.dim]
    ke = 0.5 * (j * j).sum(-1) / rho
    return (s.h ** s.dim) * torch.einsum("a,ca->", W, ke)
