// Compile-time 1-D tables of the nodal basis on [0,1]: Gauss-Legendre rule,
// Gauss-Lobatto nodes, Lagrange values and derivatives.  Evaluated by the
// compiler, so kernels index them with unrolled loop counters and the
// entries become instruction literals instead of memory reads.
//
// Gauss points: Newton on P_n from the asymptotic guess
// cos(pi (i + 3/4) / (n + 1/2)); weights 2 / ((1 - x^2) P_n'(x)^2).
// Lobatto interior nodes: Newton on P'_{n-1} (second derivative from the
// Legendre equation) from the Chebyshev-Lobatto guess cos(pi i / (n - 1)).
#pragma once

namespace dgwm {
namespace ct {

constexpr double abs_(double x) { return x < 0 ? -x : x; }

// cos on [0, pi] by its Taylor series (only used for starting guesses)
constexpr double cos_(double x) {
  double term = 1.0, sum = 1.0;
  for (int k = 1; k < 40; ++k) {
    term *= -x * x / ((2.0 * k - 1.0) * (2.0 * k));
    sum += term;
  }
  return sum;
}

constexpr double kPi = 3.14159265358979323846;

// P_n(x) and P_n'(x), |x| < 1
constexpr void legendre(int n, double x, double& p, double& dp) {
  double p0 = 1.0, p1 = x;
  if (n == 0) {
    p = 1.0;
    dp = 0.0;
    return;
  }
  for (int k = 2; k <= n; ++k) {
    const double pk = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
    p0 = p1;
    p1 = pk;
  }
  p = p1;
  dp = n * (x * p1 - p0) / (x * x - 1.0);
}

// Lagrange basis through nodes x[0..n): values and derivatives at t
template <int N>
constexpr void lagrange(const double (&x)[N], double t, double (&v)[N], double (&d)[N]) {
  for (int i = 0; i < N; ++i) {
    double den = 1.0, num = 1.0;
    for (int j = 0; j < N; ++j)
      if (j != i) {
        den *= x[i] - x[j];
        num *= t - x[j];
      }
    v[i] = num / den;
    double s = 0.0;
    for (int k = 0; k < N; ++k) {
      if (k == i) continue;
      double pr = 1.0;
      for (int j = 0; j < N; ++j)
        if (j != i && j != k) pr *= t - x[j];
      s += pr;
    }
    d[i] = s / den;
  }
}

template <int NQ>
struct Gauss {
  double g[NQ], w[NQ];
  constexpr Gauss() : g{}, w{} {
    double xs[NQ] = {}, ws[NQ] = {};
    for (int i = 0; i < NQ; ++i) {
      double x = cos_(kPi * (i + 0.75) / (NQ + 0.5));
      for (int it = 0; it < 100; ++it) {
        double p = 0, dp = 0;
        legendre(NQ, x, p, dp);
        const double dx = p / dp;
        x -= dx;
        if (abs_(dx) < 1e-17) break;
      }
      double p = 0, dp = 0;
      legendre(NQ, x, p, dp);
      xs[i] = x;
      ws[i] = 2.0 / ((1.0 - x * x) * dp * dp);
    }
    // xs descends; map to [0, 1] ascending
    for (int i = 0; i < NQ; ++i) {
      g[i] = 0.5 * (1.0 - xs[i]);
      w[i] = 0.5 * ws[i];
    }
  }
};

template <int NP>
struct Lobatto {
  double x[NP];
  constexpr Lobatto() : x{} {
    const int n = NP - 1;  // interior nodes are the roots of P_n'
    double r[NP] = {};
    r[0] = -1.0;
    r[NP - 1] = 1.0;
    for (int i = 1; i < NP - 1; ++i) {
      double t = -cos_(kPi * i / n);
      for (int it = 0; it < 100; ++it) {
        double p = 0, dp = 0;
        legendre(n, t, p, dp);
        const double d2 = (2.0 * t * dp - n * (n + 1.0) * p) / (1.0 - t * t);
        const double dt = dp / d2;
        t -= dt;
        if (abs_(dt) < 1e-17) break;
      }
      r[i] = t;
    }
    for (int i = 0; i < NP; ++i) x[i] = 0.5 * (r[i] + 1.0);
  }
};

// Tables of the NP-node Lobatto basis against the NQ-point Gauss rule:
//   S[q][i] = N_i(g_q), Sd[q][i] = N_i'(g_q), D[q][r] = L_r'(g_q) (Lagrange
//   through the Gauss points), w, g, nd0[i] = N_i'(0), nd1[i] = N_i'(1),
//   E0[q] = L_q(0), E1[q] = L_q(1): the values at the two ends of the
//   polynomial through NQ samples at the Gauss points (exact extrapolation of
//   any polynomial of degree < NQ to xi = 0 and xi = 1).
template <int NP, int NQ>
struct Tab {
  double S[NQ][NP], Sd[NQ][NP], D[NQ][NQ], w[NQ], g[NQ], nd0[NP], nd1[NP], E0[NQ], E1[NQ];
  constexpr Tab() : S{}, Sd{}, D{}, w{}, g{}, nd0{}, nd1{}, E0{}, E1{} {
    const Gauss<NQ> G;
    const Lobatto<NP> L;
    for (int q = 0; q < NQ; ++q) {
      g[q] = G.g[q];
      w[q] = G.w[q];
    }
    for (int q = 0; q < NQ; ++q) {
      double v[NP] = {}, d[NP] = {};
      lagrange(L.x, g[q], v, d);
      for (int i = 0; i < NP; ++i) {
        S[q][i] = v[i];
        Sd[q][i] = d[i];
      }
      double vq[NQ] = {}, dq[NQ] = {};
      lagrange(g, g[q], vq, dq);
      for (int r = 0; r < NQ; ++r) D[q][r] = dq[r];
    }
    double v[NP] = {}, d[NP] = {};
    lagrange(L.x, 0.0, v, d);
    for (int i = 0; i < NP; ++i) nd0[i] = d[i];
    lagrange(L.x, 1.0, v, d);
    for (int i = 0; i < NP; ++i) nd1[i] = d[i];
    double e[NQ] = {}, de[NQ] = {};
    lagrange(g, 0.0, e, de);
    for (int q = 0; q < NQ; ++q) E0[q] = e[q];
    lagrange(g, 1.0, e, de);
    for (int q = 0; q < NQ; ++q) E1[q] = e[q];
  }
};

template <int NP, int NQ>
inline constexpr Tab<NP, NQ> tab{};

template <int NP>
inline constexpr Lobatto<NP> lobatto{};

// Matrix views for the sweeps: at(m, n) is entry (m, n) of an MO x NI matrix.
template <int NP, int NQ>
struct MatS {  // N_i(g_q): rows q, columns i
  static constexpr double at(int m, int n) { return tab<NP, NQ>.S[m][n]; }
};
template <int NP, int NQ>
struct MatSd {
  static constexpr double at(int m, int n) { return tab<NP, NQ>.Sd[m][n]; }
};
template <int NP, int NQ>
struct MatD {  // collocation derivative through the Gauss points
  static constexpr double at(int m, int n) { return tab<NP, NQ>.D[m][n]; }
};

}  // namespace ct
}  // namespace dgwm
