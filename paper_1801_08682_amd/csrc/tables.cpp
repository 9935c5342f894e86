// Host construction of the 1D Gauss-Legendre nodal operators (see tables.hpp).
#include "tables.hpp"

#include <cmath>

namespace adg {

namespace {

// Legendre P_n(x) and P_n'(x) on [-1, 1] by the three-term recurrence.
void legendre(int n, double x, double* p, double* dp) {
  double p0 = 1.0, p1 = x;
  if (n == 0) { *p = 1.0; *dp = 0.0; return; }
  for (int k = 2; k <= n; ++k) {
    const double pk = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
    p0 = p1;
    p1 = pk;
  }
  *p = p1;
  *dp = n * (x * p1 - p0) / (x * x - 1.0);
}

// Gauss-Legendre nodes/weights on [-1, 1]: Newton from the Chebyshev-like
// initial guess cos(pi (k + 3/4) / (n + 1/2)); w = 2 / ((1 - x^2) P_n'(x)^2).
void gauss_legendre(int n, std::vector<double>* z, std::vector<double>* om) {
  z->assign(n, 0.0);
  om->assign(n, 0.0);
  for (int k = 0; k < n; ++k) {
    double x = std::cos(M_PI * (k + 0.75) / (n + 0.5));
    double p = 0, dp = 1;
    for (int it = 0; it < 100; ++it) {
      legendre(n, x, &p, &dp);
      const double dx = p / dp;
      x -= dx;
      if (std::fabs(dx) < 1e-17) break;
    }
    legendre(n, x, &p, &dp);
    // nodes ascending
    (*z)[n - 1 - k] = x;
    (*om)[n - 1 - k] = 2.0 / ((1.0 - x * x) * dp * dp);
  }
}

// Lagrange basis values at x from the barycentric weights lam.
void lagrange_at(const std::vector<double>& xi, const std::vector<double>& lam, double x,
                 double* out) {
  const int n = (int)xi.size();
  for (int j = 0; j < n; ++j) {
    if (x == xi[j]) {
      for (int k = 0; k < n; ++k) out[k] = (k == j) ? 1.0 : 0.0;
      return;
    }
  }
  double s = 0.0;
  for (int j = 0; j < n; ++j) s += lam[j] / (x - xi[j]);
  for (int j = 0; j < n; ++j) out[j] = (lam[j] / (x - xi[j])) / s;
}

// Solve A X = B (A n x n, B n x n, row-major) by Gaussian elimination with
// partial pivoting.  Returns false for a singular A.
bool solve(int n, std::vector<double> A, std::vector<double> B, std::vector<double>* X) {
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(A[r * n + c]) > std::fabs(A[piv * n + c])) piv = r;
    if (A[piv * n + c] == 0.0) return false;
    if (piv != c)
      for (int k = 0; k < n; ++k) {
        std::swap(A[c * n + k], A[piv * n + k]);
        std::swap(B[c * n + k], B[piv * n + k]);
      }
    for (int r = c + 1; r < n; ++r) {
      const double f = A[r * n + c] / A[c * n + c];
      for (int k = c; k < n; ++k) A[r * n + k] -= f * A[c * n + k];
      for (int k = 0; k < n; ++k) B[r * n + k] -= f * B[c * n + k];
    }
  }
  X->assign(n * n, 0.0);
  for (int k = 0; k < n; ++k)
    for (int r = n - 1; r >= 0; --r) {
      double s = B[r * n + k];
      for (int c = r + 1; c < n; ++c) s -= A[r * n + c] * (*X)[c * n + k];
      (*X)[r * n + k] = s / A[r * n + r];
    }
  return true;
}

}  // namespace

bool build_tables(int n, HostTables* t) {
  if (n < 1 || n > 16) return false;
  t->n = n;
  std::vector<double> z, om;
  gauss_legendre(n, &z, &om);
  t->xi.resize(n);
  t->w.resize(n);
  for (int k = 0; k < n; ++k) {
    t->xi[k] = 0.5 * (1.0 + z[k]);
    t->w[k] = 0.5 * om[k];
  }
  if (n == 1) { t->xi[0] = 0.5; t->w[0] = 1.0; }
  // barycentric weights
  std::vector<double> lam(n, 1.0);
  for (int j = 0; j < n; ++j)
    for (int k = 0; k < n; ++k)
      if (k != j) lam[j] /= (t->xi[j] - t->xi[k]);
  // derivative matrix, rows summing to zero
  t->D.assign(n * n, 0.0);
  for (int k = 0; k < n; ++k) {
    double diag = 0.0;
    for (int j = 0; j < n; ++j) {
      if (j == k) continue;
      const double v = (lam[j] / lam[k]) / (t->xi[k] - t->xi[j]);
      t->D[k * n + j] = v;
      diag -= v;
    }
    t->D[k * n + k] = diag;
  }
  t->FL.resize(n);
  t->FR.resize(n);
  lagrange_at(t->xi, lam, 0.0, t->FL.data());
  lagrange_at(t->xi, lam, 1.0, t->FR.data());
  // K1 and P = K1^-1 diag(w)
  std::vector<double> K1(n * n), W(n * n, 0.0);
  for (int k = 0; k < n; ++k) {
    W[k * n + k] = t->w[k];
    for (int l = 0; l < n; ++l) K1[k * n + l] = t->FR[k] * t->FR[l] - t->w[l] * t->D[l * n + k];
  }
  if (!solve(n, K1, W, &t->P)) return false;
  t->Kv.resize(n * n);
  for (int a = 0; a < n; ++a)
    for (int j = 0; j < n; ++j) t->Kv[a * n + j] = t->w[j] * t->D[j * n + a] / t->w[a];
  t->LL.resize(n);
  t->LR.resize(n);
  for (int k = 0; k < n; ++k) {
    t->LL[k] = t->FL[k] / t->w[k];
    t->LR[k] = t->FR[k] / t->w[k];
  }
  // subcell averages: Pi[s][j] = sum_q w_q phi_j((s + xi_q) / S)
  const int S = 2 * n - 1;
  t->S = S;
  t->Pi.assign(S * n, 0.0);
  std::vector<double> phi(n);
  for (int sc = 0; sc < S; ++sc)
    for (int q = 0; q < n; ++q) {
      lagrange_at(t->xi, lam, (sc + t->xi[q]) / S, phi.data());
      for (int j = 0; j < n; ++j) t->Pi[sc * n + j] += t->w[q] * phi[j];
    }
  // least-squares reconstruction Rc = (Pi^T Pi)^-1 Pi^T
  std::vector<double> A(n * n, 0.0), I(n * n, 0.0), Ainv;
  for (int a = 0; a < n; ++a) {
    I[a * n + a] = 1.0;
    for (int b = 0; b < n; ++b)
      for (int sc = 0; sc < S; ++sc) A[a * n + b] += t->Pi[sc * n + a] * t->Pi[sc * n + b];
  }
  if (!solve(n, A, I, &Ainv)) return false;
  t->Rc.assign(n * S, 0.0);
  for (int a = 0; a < n; ++a)
    for (int sc = 0; sc < S; ++sc)
      for (int b = 0; b < n; ++b) t->Rc[a * S + sc] += Ainv[a * n + b] * t->Pi[sc * n + b];
  return true;
}

}  // namespace adg
