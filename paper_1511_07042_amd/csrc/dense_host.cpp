// Setup-time dense generalized symmetric-definite eigensolver for the
// level-0 problem A_0 x = lambda M_0 x (the "direct eigensolve" on the
// coarsest level, Alg. 2 step 1).  Method (Golub & Van Loan, Matrix
// Computations, Sec. 8.7 and 8.5): Cholesky M = L L^T, reduction to
// C = L^-1 A L^-T, cyclic Jacobi on C, back-transformation x = L^-T q.
#include <algorithm>
#include <cmath>
#include <numeric>

#include "bmg_internal.h"

namespace bmg {

int dense_sygv(int n, const std::vector<double>& A, const std::vector<double>& M,
               std::vector<double>& lam, std::vector<double>& X) {
  auto at = [n](std::vector<double>& v, int i, int j) -> double& { return v[size_t(i) * n + j]; };
  // Cholesky (lower)
  std::vector<double> L(size_t(n) * n, 0.0);
  for (int j = 0; j < n; ++j) {
    double d = M[size_t(j) * n + j];
    for (int k = 0; k < j; ++k) d -= at(L, j, k) * at(L, j, k);
    BMG_CHECK(d > 0, "mass matrix of level 0 is not positive definite");
    const double ljj = std::sqrt(d);
    at(L, j, j) = ljj;
    for (int i = j + 1; i < n; ++i) {
      double s = M[size_t(i) * n + j];
      for (int k = 0; k < j; ++k) s -= at(L, i, k) * at(L, j, k);
      at(L, i, j) = s / ljj;
    }
  }
  // B = L^-1 A (forward substitution per column), C = B L^-T = (L^-1 B^T)^T
  std::vector<double> B(A), C(size_t(n) * n);
  for (int c = 0; c < n; ++c)
    for (int i = 0; i < n; ++i) {
      double s = at(B, i, c);
      for (int k = 0; k < i; ++k) s -= at(L, i, k) * at(B, k, c);
      at(B, i, c) = s / at(L, i, i);
    }
  for (int r = 0; r < n; ++r)
    for (int i = 0; i < n; ++i) {
      double s = at(B, r, i);
      for (int k = 0; k < i; ++k) s -= at(L, i, k) * at(C, r, k);
      at(C, r, i) = s / at(L, i, i);
    }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < i; ++j) at(C, i, j) = at(C, j, i) = 0.5 * (at(C, i, j) + at(C, j, i));
  // cyclic Jacobi
  std::vector<double> V(size_t(n) * n, 0.0);
  for (int i = 0; i < n; ++i) at(V, i, i) = 1.0;
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        const double v = at(C, i, j) * at(C, i, j);
        tot += v;
        if (i != j) off += v;
      }
    if (off <= 1e-32 * tot || off == 0.0) break;
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = at(C, p, q);
        if (apq == 0.0) continue;
        const double tau = (at(C, q, q) - at(C, p, p)) / (2.0 * apq);
        const double t = (tau >= 0 ? 1.0 : -1.0) / (std::fabs(tau) + std::sqrt(1.0 + tau * tau));
        const double c = 1.0 / std::sqrt(1.0 + t * t), s = t * c;
        for (int k = 0; k < n; ++k) {  // C <- C J
          const double ckp = at(C, k, p), ckq = at(C, k, q);
          at(C, k, p) = c * ckp - s * ckq;
          at(C, k, q) = s * ckp + c * ckq;
        }
        for (int k = 0; k < n; ++k) {  // C <- J^T C
          const double cpk = at(C, p, k), cqk = at(C, q, k);
          at(C, p, k) = c * cpk - s * cqk;
          at(C, q, k) = s * cpk + c * cqk;
        }
        at(C, p, q) = at(C, q, p) = 0.0;
        for (int k = 0; k < n; ++k) {  // V <- V J
          const double vkp = at(V, k, p), vkq = at(V, k, q);
          at(V, k, p) = c * vkp - s * vkq;
          at(V, k, q) = s * vkp + c * vkq;
        }
      }
  }
  std::vector<int> ord(n);
  std::iota(ord.begin(), ord.end(), 0);
  std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return at(C, a, a) < at(C, b, b); });
  lam.resize(n);
  X.assign(size_t(n) * n, 0.0);
  for (int j = 0; j < n; ++j) {
    lam[j] = at(C, ord[j], ord[j]);
    // x = L^-T v (back substitution)
    for (int i = n - 1; i >= 0; --i) {
      double s = at(V, i, ord[j]);
      for (int k = i + 1; k < n; ++k) s -= at(L, k, i) * at(X, k, j);
      at(X, i, j) = s / at(L, i, i);
    }
  }
  return BMG_OK;
}

}  // namespace bmg
