"""1D nodal operators on the unit interval for the Gauss-Legendre Lagrange basis.

Oracle (test infrastructure only; see the package docstring).

Sec. 3 of the paper spans the solution per cell by a tensor-product Lagrange
basis on Gauss-Legendre collocation points and states that this basis gives a
quadrature-free formulation with sparse operators.  The paper does not print
the operators; the ones below follow from its weak forms:

* Eq. (3), the cell-local space-time problem, tested with theta_k(tau) phi_a(x)
  and integrated by parts in time with the cell state at tau = 0 as upwind
  value, gives the time matrix ``K1`` and ``P = K1^-1 diag(w)``;
* Eq. (2), the update, gives the volume operator ``Kv`` (from the gradient of
  the test function) and the lifting vectors ``LL``, ``LR`` (from the face
  integral), once divided by the diagonal GL mass matrix.

All tables are float64 numpy arrays.  Nodes and weights come from numpy's
Gauss-Legendre routine; everything else is computed here from its definition.
"""

from dataclasses import dataclass

import numpy as np


def gauss_legendre_unit(n):
    """GL nodes xi and weights w on [0, 1] (n points, exact to degree 2n-1).

    Library primitive (numpy.polynomial.legendre.leggauss) mapped from [-1, 1].
    """
    z, om = np.polynomial.legendre.leggauss(n)
    return 0.5 * (1.0 + z), 0.5 * om


def barycentric_weights(xi):
    """lambda_j = 1 / prod_{k != j} (xi_j - xi_k)  (barycentric Lagrange form)."""
    n = len(xi)
    lam = np.ones(n)
    for j in range(n):
        for k in range(n):
            if k != j:
                lam[j] /= (xi[j] - xi[k])
    return lam


def lagrange_values(xi, lam, x):
    """phi_j(x) for all j, second barycentric formula; exact at the nodes."""
    n = len(xi)
    diff = x - xi
    hit = np.nonzero(diff == 0.0)[0]
    if len(hit):
        out = np.zeros(n)
        out[hit[0]] = 1.0
        return out
    t = lam / diff
    return t / t.sum()


def derivative_matrix(xi, lam):
    """D[k][j] = phi_j'(xi_k).

    Off-diagonal: (lam_j / lam_k) / (xi_k - xi_j); the diagonal makes each row
    sum to zero (the derivative of the constant 1 vanishes).
    """
    n = len(xi)
    D = np.zeros((n, n))
    for k in range(n):
        for j in range(n):
            if j != k:
                D[k, j] = (lam[j] / lam[k]) / (xi[k] - xi[j])
        D[k, k] = -D[k].sum()
    return D


@dataclass(frozen=True)
class Tables:
    order: int          # polynomial degree N (the paper's p)
    xi: np.ndarray      # GL nodes on [0,1]
    w: np.ndarray       # GL weights on [0,1], sum 1
    D: np.ndarray       # D[k][j] = phi_j'(xi_k)
    FL: np.ndarray      # phi_j(0)
    FR: np.ndarray      # phi_j(1)
    K1: np.ndarray      # time stiffness with upwind value at tau=0
    P: np.ndarray       # K1^-1 diag(w)
    Kv: np.ndarray      # volume operator, Kv[a][j] = w_j D[j][a] / w_a
    LL: np.ndarray      # FL / w  (lift of the left-face flux)
    LR: np.ndarray      # FR / w  (lift of the right-face flux)

    @property
    def n(self):
        return self.order + 1


def make_tables(order):
    """All 1D operators for degree ``order`` (n = order + 1 GL nodes).

    K1[k][l] = theta_k(1) theta_l(1) - int_0^1 theta_k' theta_l dtau
             = FR_k FR_l - w_l D[l][k]           (GL is exact for this degree)
    From the time-tested Eq. (3):  K1 q = FL u - dt diag(w) rhs, hence
    q = (K1^-1 FL) u - dt P rhs with K1^-1 FL = 1 (K1 applied to ones is FL).
    """
    n = order + 1
    xi, w = gauss_legendre_unit(n)
    lam = barycentric_weights(xi)
    D = derivative_matrix(xi, lam)
    FL = lagrange_values(xi, lam, 0.0)
    FR = lagrange_values(xi, lam, 1.0)
    K1 = np.outer(FR, FR) - (w[:, None] * D).T
    P = np.linalg.solve(K1, np.diag(w))
    Kv = (w[:, None] * D).T / w[:, None]
    return Tables(order=order, xi=xi, w=w, D=D, FL=FL, FR=FR, K1=K1, P=P,
                  Kv=Kv, LL=FL / w, LR=FR / w)
