"""Conservative fluxes F_i(Q) and directional wave speeds of the four PDEs.

Oracle (test infrastructure only).

Eq. (1) of the paper with B_i = 0, S = 0, no point sources (the simplification
the paper itself makes in Sec. 3):  dQ/dt + sum_i d/dx_i F_i(Q) = 0.

* Euler (Sec. 7, the paper's benchmark PDE): Q = (rho, j, E),
  F_i = (j_i, j_i j / rho + p e_i, j_i (E + p) / rho),
  p = (gamma - 1) (E - |j|^2 / (2 rho)), gamma - 1 = 0.4 in the paper.
  The wave speed along axis i is |u_i| + sqrt(gamma p / rho), the largest
  eigenvalue modulus of dF_i/dQ.
* Linear advection: F_i = a_i q, speed |a_i|.
* Linear acoustics (rho_0 = 1, bulk modulus c^2 per cell): Q = (p, u),
  F_i = (c^2 u_i, p e_i), speed c.
* Linear elasticity (velocity-stress form, per cell rho, lambda, mu):
  Q = (v, sigma) with sigma in Voigt order (11, 22, 33, 12, 23, 13) in 3D and
  (11, 22, 12) in 2D; F_i(v_k) = -sigma_ik / rho,
  F_i(sigma_kl) = -(lambda delta_kl v_i + mu (delta_ik v_l + delta_il v_k)),
  speed sqrt((lambda + 2 mu) / rho).

Material coefficients are constant per cell and enter in conservative flux
form (the paper routes material jumps through B_i, which it neglects).

Every function takes ``q`` with the variables on the last axis and a
per-cell parameter tensor ``par`` broadcastable to ``q.shape[:-1] + (npar,)``.
"""

import torch

ADVECTION, EULER, ELASTIC, ACOUSTIC = 0, 1, 2, 3
NAMES = {ADVECTION: "advection", EULER: "euler", ELASTIC: "elastic",
         ACOUSTIC: "acoustic"}


def _voigt(d):
    """(k, l) pairs of the stress components in Voigt order."""
    if d == 3:
        return [(0, 0), (1, 1), (2, 2), (0, 1), (1, 2), (0, 2)]
    return [(0, 0), (1, 1), (0, 1)]


class PDE:
    kind = None
    npar = 0          # per-cell parameters
    linear = False

    def __init__(self, d, pde_param=()):
        self.d = d
        self.pp = tuple(float(x) for x in pde_param)

    def flux(self, q, i, par):
        raise NotImplementedError

    def speed(self, q, i, par):
        raise NotImplementedError


class Advection(PDE):
    kind = ADVECTION
    linear = True

    @property
    def m(self):
        return 1

    def flux(self, q, i, par):
        return self.pp[i] * q

    def speed(self, q, i, par):
        return torch.full(q.shape[:-1], abs(self.pp[i]), dtype=q.dtype)


class Euler(PDE):
    kind = EULER

    @property
    def m(self):
        return self.d + 2

    @property
    def gamma(self):
        return self.pp[0] if self.pp else 1.4

    def pressure(self, q):
        rho = q[..., 0]
        j = q[..., 1:1 + self.d]
        E = q[..., 1 + self.d]
        return (self.gamma - 1.0) * (E - 0.5 * (j * j).sum(-1) / rho)

    def flux(self, q, i, par):
        d = self.d
        rho = q[..., 0]
        j = q[..., 1:1 + d]
        E = q[..., 1 + d]
        p = self.pressure(q)
        ui = j[..., i] / rho
        comps = [j[..., i]]
        for k in range(d):
            t = j[..., k] * ui
            if k == i:
                t = t + p
            comps.append(t)
        comps.append(ui * (E + p))
        return torch.stack(comps, -1)

    def speed(self, q, i, par):
        rho = q[..., 0]
        ui = q[..., 1 + i] / rho
        p = self.pressure(q)
        return ui.abs() + torch.sqrt(self.gamma * p / rho)


class Acoustic(PDE):
    """par[..., 0] = sound speed c of the cell."""
    kind = ACOUSTIC
    npar = 1
    linear = True

    @property
    def m(self):
        return self.d + 1

    def flux(self, q, i, par):
        c = par[..., 0]
        p = q[..., 0]
        comps = [c * c * q[..., 1 + i]]
        zero = torch.zeros_like(p)
        for k in range(self.d):
            comps.append(p if k == i else zero)
        return torch.stack(comps, -1)

    def speed(self, q, i, par):
        return par[..., 0].expand(q.shape[:-1]).clone()


class Elastic(PDE):
    """par[..., 0:3] = (rho, lambda, mu) of the cell."""
    kind = ELASTIC
    npar = 3
    linear = True

    @property
    def m(self):
        return self.d + len(_voigt(self.d))

    def flux(self, q, i, par):
        d = self.d
        rho, lam, mu = par[..., 0], par[..., 1], par[..., 2]
        v = [q[..., k] for k in range(d)]
        sig = {}
        for s, (k, l) in enumerate(_voigt(d)):
            sig[(k, l)] = q[..., d + s]
            sig[(l, k)] = q[..., d + s]
        comps = [-sig[(i, k)] / rho for k in range(d)]
        for (k, l) in _voigt(d):
            t = mu * ((v[l] if i == k else 0.0) + (v[k] if i == l else 0.0))
            if k == l:
                t = t + lam * v[i]
            comps.append(-t * torch.ones_like(v[0]))
        return torch.stack(comps, -1)

    def speed(self, q, i, par):
        rho, lam, mu = par[..., 0], par[..., 1], par[..., 2]
        return torch.sqrt((lam + 2.0 * mu) / rho).expand(q.shape[:-1]).clone()


def make_pde(kind, d, pde_param=()):
    return {ADVECTION: Advection, EULER: Euler, ELASTIC: Elastic,
            ACOUSTIC: Acoustic}[kind](d, pde_param)
