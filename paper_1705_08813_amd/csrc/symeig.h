// Host-side dense symmetric eigendecomposition (cyclic Jacobi method).
#pragma once

#include <cmath>
#include <vector>

namespace dgwm {

// A = Z diag(lam) Z^T for a symmetric n x n matrix a (row-major; destroyed).
// Cyclic Jacobi: sweep over all pairs (p, q), p < q, and zero a_pq with the
// plane rotation whose angle solves the 2 x 2 symmetric eigenproblem of rows
// and columns p, q; repeat until the off-diagonal part is below 1e-32 of the
// squared Frobenius norm (quadratic convergence once the off-diagonal part
// is small).  vt (row-major n x n) holds the eigenvectors as ROWS on return:
// vt[i][k] = Z[k][i].  Returns the number of sweeps, or -1 if 60 sweeps did
// not converge.
inline int sym_eig_jacobi(int n, std::vector<double>& a, std::vector<double>& lam, std::vector<double>& vt) {
  vt.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) vt[(size_t)i * n + i] = 1.0;
  double fro = 0.0;
  for (size_t i = 0; i < (size_t)n * n; ++i) fro += a[i] * a[i];
  int sweep = 0;
  for (; sweep < 60; ++sweep) {
    double off = 0.0;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) off += a[(size_t)p * n + q] * a[(size_t)p * n + q];
    if (off <= 1e-32 * fro || off == 0.0) break;
    for (int p = 0; p < n - 1; ++p) {
      double* ap = &a[(size_t)p * n];
      for (int q = p + 1; q < n; ++q) {
        double* aq = &a[(size_t)q * n];
        const double apq = ap[q];
        if (apq == 0.0) continue;
        const double app = ap[p], aqq = aq[q];
        if (std::fabs(apq) <= 1e-18 * (std::fabs(app) + std::fabs(aqq))) {
          ap[q] = aq[p] = 0.0;
          continue;
        }
        // t = tan(angle): smaller root of t^2 + 2 theta t - 1 = 0
        const double theta = (aqq - app) / (2.0 * apq);
        const double t = (theta >= 0.0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        // columns p, q of A <- A J; then rows by symmetry
        for (int k = 0; k < n; ++k) {
          const double akp = ap[k], akq = aq[k];  // row entries = column entries (symmetric)
          ap[k] = c * akp - s * akq;
          aq[k] = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {
          double* ak = &a[(size_t)k * n];
          ak[p] = ap[k];
          ak[q] = aq[k];
        }
        ap[p] = app - t * apq;
        aq[q] = aqq + t * apq;
        ap[q] = aq[p] = 0.0;
        double* vp = &vt[(size_t)p * n];
        double* vq = &vt[(size_t)q * n];
        for (int k = 0; k < n; ++k) {
          const double x = vp[k], y = vq[k];
          vp[k] = c * x - s * y;
          vq[k] = s * x + c * y;
        }
      }
    }
  }
  lam.resize(n);
  for (int i = 0; i < n; ++i) lam[i] = a[(size_t)i * n + i];
  return sweep < 60 ? sweep : -1;
}

}  // namespace dgwm
