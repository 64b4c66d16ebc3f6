// Host-side 1-D quadrature rules and nodal-basis tables.
//
// Gauss-Legendre points are the roots of the Legendre polynomial P_n, found
// by Newton's method from the asymptotic (Tricomi) initial guess; weights
// w = 2 / ((1 - t^2) P_n'(t)^2).  Gauss-Lobatto nodes are the end points and
// the roots of P_{n-1}'.  The nodal basis is evaluated in barycentric form.
// Everything is mapped to the reference interval [0,1].
#include <algorithm>
#include <cmath>
#include <vector>

#include "dgwm_internal.h"

namespace dgwm {

namespace {

// P_n(t), P_n'(t) by the three-term recurrence.
void legendre_pd(int n, double t, double& p, double& dp) {
  double pm1 = 1.0, pc = t;
  if (n == 0) {
    p = 1.0;
    dp = 0.0;
    return;
  }
  for (int k = 1; k < n; ++k) {
    double pn = ((2 * k + 1) * t * pc - k * pm1) / (k + 1);
    pm1 = pc;
    pc = pn;
  }
  p = pc;
  dp = n * (t * pc - pm1) / (t * t - 1.0);
}

// Barycentric weights of a node set.
std::vector<double> bary_weights(const double* x, int n) {
  std::vector<double> lam(n, 1.0);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j)
      if (j != i) lam[i] /= (x[i] - x[j]);
  return lam;
}

// Values and first derivatives of the Lagrange basis through x at t.
void lagrange_eval(const double* x, int n, double t, double* v, double* d) {
  std::vector<double> lam = bary_weights(x, n);
  for (int i = 0; i < n; ++i) {
    if (t == x[i]) {
      // at a node: cardinal values; N_j'(x_i) = (lam_j/lam_i)/(x_i - x_j),
      // N_i'(x_i) = sum_{j != i} 1/(x_i - x_j)
      double s = 0.0;
      for (int j = 0; j < n; ++j) {
        v[j] = (j == i) ? 1.0 : 0.0;
        if (j == i) continue;
        d[j] = lam[j] / lam[i] / (x[i] - x[j]);
        s += 1.0 / (x[i] - x[j]);
      }
      d[i] = s;
      return;
    }
  }
  // l(t) = prod (t - x_j); N_i = l lam_i / (t - x_i);
  // N_i' = N_i * (sum_{j != i} 1/(t - x_j))
  double l = 1.0;
  for (int j = 0; j < n; ++j) l *= (t - x[j]);
  double sall = 0.0;
  for (int j = 0; j < n; ++j) sall += 1.0 / (t - x[j]);
  for (int i = 0; i < n; ++i) {
    v[i] = l * lam[i] / (t - x[i]);
    d[i] = v[i] * (sall - 1.0 / (t - x[i]));
  }
}

}  // namespace

void gauss_rule(int n, double* x, double* w) {
  for (int i = 1; i <= n; ++i) {
    // Tricomi guess for the i-th root (descending)
    double th = M_PI * (4.0 * i - 1.0) / (4.0 * n + 2.0);
    double t = (1.0 - (n - 1.0) / (8.0 * n * n * n)) * std::cos(th);
    double p, dp;
    for (int it = 0; it < 50; ++it) {
      legendre_pd(n, t, p, dp);
      double dt = p / dp;
      t -= dt;
      if (std::fabs(dt) <= 1e-16) break;
    }
    legendre_pd(n, t, p, dp);
    int k = n - i;  // ascending
    x[k] = 0.5 * (1.0 + t);
    w[k] = 1.0 / ((1.0 - t * t) * dp * dp);  // half of the [-1,1] weight
  }
}

void lobatto_nodes(int n, double* x) {
  x[0] = 0.0;
  x[n - 1] = 1.0;
  int m = n - 1;  // roots of P_m'
  for (int i = 1; i < m; ++i) {
    double t = -std::cos(M_PI * i / m);
    for (int it = 0; it < 60; ++it) {
      // q(t) = P_m'(t); q'(t) from (1-t^2) P'' = 2 t P' - m(m+1) P
      double p, dp;
      legendre_pd(m, t, p, dp);
      double d2p = (2.0 * t * dp - m * (m + 1.0) * p) / (1.0 - t * t);
      double dt = dp / d2p;
      t -= dt;
      if (std::fabs(dt) <= 1e-16) break;
    }
    x[i] = 0.5 * (1.0 + t);
  }
}

// Fill the TabLayout of (np, nq, nqy).
void fill_tables(int np, int nq, int nqy, double* out) {
  const TabLayout L = tab_layout(np, nq, nqy);
  double gl[kMaxP];
  lobatto_nodes(np, gl);
  auto rule = [&](int n, int oS, int oSd, int oD, int ow, int og) {
    double g[kMaxQ], w[kMaxQ], v[kMaxQ], d[kMaxQ];
    gauss_rule(n, g, w);
    for (int q = 0; q < n; ++q) {
      lagrange_eval(gl, np, g[q], v, d);
      for (int i = 0; i < np; ++i) {
        out[oS + q * np + i] = v[i];
        out[oSd + q * np + i] = d[i];
      }
      // collocation derivative through the Gauss points themselves
      lagrange_eval(g, n, g[q], v, d);
      for (int r = 0; r < n; ++r) out[oD + q * n + r] = d[r];
      out[ow + q] = w[q];
      out[og + q] = g[q];
    }
  };
  rule(nq, L.S, L.Sd, L.D, L.w, L.g);
  rule(nqy, L.Sy, L.Sdy, L.Dy, L.wy, L.gy);
  double v[kMaxP], d[kMaxP];
  lagrange_eval(gl, np, 0.0, v, d);
  for (int i = 0; i < np; ++i) out[L.nd0 + i] = d[i];
  lagrange_eval(gl, np, 1.0, v, d);
  for (int i = 0; i < np; ++i) out[L.nd1 + i] = d[i];
  for (int i = 0; i < np; ++i) out[L.gl + i] = gl[i];
}

void fill_poisson_ops(int np, int nq, double* out) {
  const PoiOps o = poi_ops(np);
  double gl[kMaxP], g[kMaxQ], w[kMaxQ], v[kMaxQ][kMaxP], d[kMaxQ][kMaxP];
  lobatto_nodes(np, gl);
  gauss_rule(nq, g, w);
  for (int q = 0; q < nq; ++q) lagrange_eval(gl, np, g[q], v[q], d[q]);
  for (int i = 0; i < np; ++i)
    for (int j = 0; j < np; ++j) {
      double m = 0, k = 0;
      for (int q = 0; q < nq; ++q) {
        m += w[q] * v[q][i] * v[q][j];
        k += w[q] * d[q][i] * d[q][j];
      }
      out[o.M + i * np + j] = m;
      out[o.K + i * np + j] = k;
    }
  double v0[kMaxP], d0[kMaxP];
  lagrange_eval(gl, np, 0.0, v0, d0);
  for (int i = 0; i < np; ++i) out[o.nd0 + i] = d0[i];
  lagrange_eval(gl, np, 1.0, v0, d0);
  for (int i = 0; i < np; ++i) out[o.nd1 + i] = d0[i];
  float* f = reinterpret_cast<float*>(out + o.f32);
  for (int i = 0; i < o.n; ++i) f[i] = (float)out[i];
}

// van Driest's law at the support points y+_i = 0, 5, 11, 24, 59, 144, 361,
// 946, 2517 (the locations of the paper's Table tab:psi): composite 12-point
// Gauss-Legendre on unit panels up to 64, then panels of 10 % of the abscissa
// (the integrand is analytic, so every panel is exact to rounding).
void vandriest_table(double kappa, double A_plus, VdTable& t) {
  static const double ys[VdTable::N] = {0.0, 5.0, 11.0, 24.0, 59.0, 144.0, 361.0, 946.0, 2517.0};
  double g[kMaxQ + 4], w[kMaxQ + 4];
  gauss_rule(12, g, w);
  auto f = [&](double s) {
    const double m = 2.0 * kappa * s * (-std::expm1(-s / A_plus));
    return 2.0 / (1.0 + std::sqrt(1.0 + m * m));
  };
  double acc = 0.0, a = 0.0;
  for (int i = 0; i < VdTable::N; ++i) {
    while (a < ys[i]) {
      const double width = a < 64.0 ? 1.0 : 0.1 * a;
      const double b = std::min(a + width, ys[i]);
      double sum = 0.0;
      for (int q = 0; q < 12; ++q) sum += w[q] * f(a + (b - a) * g[q]);
      acc += (b - a) * sum;
      a = b;
    }
    t.y[i] = ys[i];
    t.psi[i] = acc;
  }
}

}  // namespace dgwm
