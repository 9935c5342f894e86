// 1D nodal operators for the Gauss-Legendre Lagrange basis on [0, 1].
//
// Sec. 3 of the paper spans each cell's solution by a tensor-product Lagrange
// basis on Gauss-Legendre points and solves the space-time predictor with
// quadrature-free operators.  With n = N + 1 nodes xi_k and weights w_k:
//   D[k][j]  = phi_j'(xi_k)                      derivative matrix
//   FL, FR   = phi_j(0), phi_j(1)                face evaluation
//   K1[k][l] = FR_k FR_l - w_l D[l][k]           time matrix, upwind at tau = 0
//   P        = K1^-1 diag(w)                     Picard time operator
//   Kv[a][j] = w_j D[j][a] / w_a                 volume term of the update
//   LL, LR   = FL / w, FR / w                    face lifting
// and, for the limiter's subcell patches (S = 2N + 1 = 2n - 1 subcells per
// axis; Sec. 3 "Finite Volume limiter"):
//   Pi[s][j] = average of phi_j over subcell s     (S x n, an n-point Gauss
//                                                 rule per subcell: exact)
//   Rc = (Pi^T Pi)^-1 Pi^T                        (n x S, least squares back)
// Computed on the host in double precision; no device code here.
#pragma once

#include <vector>

namespace adg {

struct HostTables {
  int n = 0;
  std::vector<double> xi, w, D, FL, FR, P, Kv, LL, LR;   // row-major n x n where 2D
  int S = 0;
  std::vector<double> Pi, Rc;                            // S x n and n x S, row-major
};

// Returns false when n is outside [1, 16].
bool build_tables(int n, HostTables* t);

}  // namespace adg
