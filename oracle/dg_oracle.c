/*
 * dg_oracle.c -- plain FP64 CPU oracle for the enriched DG operators.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header, table or constant
 * generator with the HIP path.
 *
 * Everything is computed by the plain definition: for every cell, every
 * quadrature point and every basis function, the 3-D basis value and
 * gradient are formed directly as products of 1-D Lagrange values and
 * derivatives, and the integrals are accumulated point by point.  No sum
 * factorization, no blocking, no reordering.  Faces are handled element by
 * element (each cell evaluates both traces of each of its six faces), so
 * every output entry has exactly one writer and OpenMP over cells is safe.
 *
 * Citations refer to Krank, Kronbichler & Wall, "A multiscale approach to
 * hybrid RANS/LES wall modeling within a high-order discontinuous Galerkin
 * scheme using function enrichment" (arXiv 1705.08813):
 *   - function spaces and enrichment: Sec. 3.1, eqs. (space), (std_fe),
 *     (enrichment); l = 0 weights (one constant per component and cell);
 *   - wall coordinate y+ and nodal wall distance y_h: Sec. 3.2;
 *   - convective operator with local Lax-Friedrichs flux: Sec. 4.2;
 *   - viscous term: Sec. 4.2 eq. (viscous_multiscale), last row (LES/LES),
 *     with the adjoint sign as a parameter theta (theta = +1 symmetric
 *     interior penalty, theta = -1 the paper's nonsymmetric row) and
 *     nu_t = 0; penalty x10 on no-slip faces (Sec. 4.2);
 *   - mirror boundary values on no-slip walls: end of Sec. 4.2;
 *   - pressure Laplace operator (SIP): Sec. 4.2, Laplace term and eq. (ipflux),
 *     homogeneous Neumann data on walls;
 *   - quadrature policy: Sec. 4.4 (k+1 Gauss points linear, floor(3k/2)+1
 *     nonlinear, a larger wall-normal rule in enriched cells);
 *   - tanh grading of the channel mesh: Sec. 5.1.
 * Spalding's law is not written out in the paper (Sec. 3.2 names it as the
 * enrichment of the authors' earlier work); the implicit law used here is the
 * standard published form  y+ = U + exp(-kappa B) (exp(kappa U) - 1 - kappa U
 * - (kappa U)^2/2 - (kappa U)^3/6).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#define ORC_MAXN 16

typedef struct {
  int32_t nx, ny, nz;
  double Lx, Lz;
  double gamma;     /* tanh grading, 0 = uniform */
  double wall_amp;  /* lower-wall cosine amplitude, 0 = flat */
  int32_t k_u, k_p;
  int32_t nq_u, nq_p, nq_wn;
  int32_t enrich_lower, enrich_upper, fully_periodic;
  double nu, kappa, B;
  double ip_factor_u, ip_factor_p, wall_ip_mult, theta;
  int32_t psi_kind; /* 0: Spalding's law, 1: van Driest's law (Sec. 3.2, eq. psi) */
  double A_plus;    /* van Driest damping constant A+ */
  double yplus_off; /* > 0: the enrichment of a wall cell is off while every quadrature point of
                       the cell has y+ below this value (Sec. 3.2: 30); 0: always on */
  int32_t enrich_degree; /* tensor degree l of the enrichment weights (Sec. 3.1, eq. enrichment): 0 or 1 */
} orc_params;

/* ------------------------------------------------------------------------ */
/* 1-D polynomials                                                           */
/* ------------------------------------------------------------------------ */

/* Legendre polynomial P_n and its derivative at t in [-1,1] (three-term
 * recurrence; derivative from (1-t^2) P_n' = n (P_{n-1} - t P_n)). */
static void legendre(int n, double t, double *P, double *dP) {
  double p0 = 1.0, p1 = t;
  if (n == 0) { *P = 1.0; *dP = 0.0; return; }
  for (int m = 2; m <= n; ++m) {
    double p2 = ((2.0 * m - 1.0) * t * p1 - (m - 1.0) * p0) / m;
    p0 = p1; p1 = p2;
  }
  *P = p1;
  if (fabs(1.0 - t * t) > 1e-300)
    *dP = n * (p0 - t * p1) / (1.0 - t * t);
  else
    *dP = 0.5 * n * (n + 1.0) * (t > 0 ? 1.0 : ((n % 2) ? 1.0 : -1.0));
}

/* n-point Gauss-Legendre rule mapped to [0,1]: nodes are the roots of P_n
 * (Newton from Chebyshev guesses), weights 2/((1-t^2) P_n'(t)^2), halved. */
int orc_gauss(int n, double *x, double *w) {
  if (n < 1 || n > ORC_MAXN) return -1;
  for (int i = 0; i < n; ++i) {
    double t = cos(M_PI * (i + 0.75) / (n + 0.5));
    for (int it = 0; it < 100; ++it) {
      double P, dP;
      legendre(n, t, &P, &dP);
      double dt = P / dP;
      t -= dt;
      if (fabs(dt) < 1e-17) break;
    }
    double P, dP;
    legendre(n, t, &P, &dP);
    /* ascending order on [0,1] */
    x[n - 1 - i] = 0.5 * (t + 1.0);
    w[n - 1 - i] = 0.5 * 2.0 / ((1.0 - t * t) * dP * dP);
  }
  return 0;
}

/* n-point Gauss-Lobatto nodes on [0,1]: the two end points plus the roots of
 * P'_{n-1}; Newton on P'_{n-1} using the Legendre equation for P''. */
int orc_gauss_lobatto(int n, double *x) {
  if (n < 2 || n > ORC_MAXN) return -1;
  int k = n - 1;
  x[0] = 0.0;
  x[n - 1] = 1.0;
  for (int i = 1; i < k; ++i) {
    double t = -cos(M_PI * i / k);
    for (int it = 0; it < 100; ++it) {
      double P, dP;
      legendre(k, t, &P, &dP);
      double d2P = (2.0 * t * dP - k * (k + 1.0) * P) / (1.0 - t * t);
      double dt = dP / d2P;
      t -= dt;
      if (fabs(dt) < 1e-17) break;
    }
    x[i] = 0.5 * (t + 1.0);
  }
  return 0;
}

/* Lagrange basis through `nodes` evaluated at t: values and derivatives,
 * straight from the product formula. */
void orc_lagrange(int n, const double *nodes, double t, double *val, double *der) {
  for (int i = 0; i < n; ++i) {
    double v = 1.0;
    for (int j = 0; j < n; ++j)
      if (j != i) v *= (t - nodes[j]) / (nodes[i] - nodes[j]);
    val[i] = v;
    double d = 0.0;
    for (int l = 0; l < n; ++l) {
      if (l == i) continue;
      double p = 1.0 / (nodes[i] - nodes[l]);
      for (int j = 0; j < n; ++j)
        if (j != i && j != l) p *= (t - nodes[j]) / (nodes[i] - nodes[j]);
      d += p;
    }
    der[i] = d;
  }
}

/* ------------------------------------------------------------------------ */
/* Spalding's law (implicit), solved for U given y+                           */
/* ------------------------------------------------------------------------ */

static double spalding_f(double U, double yp, double kappa, double B) {
  double x = kappa * U;
  if (x > 700.0) return INFINITY;
  return U + exp(-kappa * B) * (exp(x) - 1.0 - x - 0.5 * x * x - x * x * x / 6.0) - yp;
}

static double spalding_df(double U, double kappa, double B) {
  double x = kappa * U;
  if (x > 700.0) return INFINITY;
  return 1.0 + kappa * exp(-kappa * B) * (exp(x) - 1.0 - x - 0.5 * x * x);
}

/* Safeguarded Newton on [0, y+]: f(0) = -y+ <= 0 and f(y+) >= 0 because the
 * bracketed series is non-negative for U >= 0.  Steps that leave the bracket
 * are replaced by bisection.  Returns U and dU/dy+. */
int orc_spalding(double yp, double kappa, double B, double *U_out, double *dU_out) {
  if (!(yp >= 0.0) || !isfinite(yp)) return -1;
  if (yp == 0.0) { *U_out = 0.0; *dU_out = 1.0; return 0; }
  double lo = 0.0, hi = yp;
  double U = (yp < 10.0) ? yp : log(yp) / kappa + B;
  if (U > hi) U = hi;
  for (int it = 0; it < 200; ++it) {
    double f = spalding_f(U, yp, kappa, B);
    if (f == 0.0) break;
    if (f > 0) hi = U; else lo = U;
    double Un = U - f / spalding_df(U, kappa, B);
    if (!(Un >= lo && Un <= hi)) Un = 0.5 * (lo + hi);
    double dU = fabs(Un - U);
    U = Un;
    if (dU <= 4e-16 * fmax(1.0, U)) break;
  }
  *U_out = U;
  *dU_out = 1.0 / spalding_df(U, kappa, B);
  return 0;
}

/* van Driest's law (Sec. 3.2, eq. psi): U(y+) = int_0^{y+} f, with
 * f(s) = 2 / (1 + sqrt(1 + (2 kappa s (1 - exp(-s/A+)))^2)), dU/dy+ = f(y+).
 * Composite Gauss-Legendre from 0 (no tabulation): 12-point panels of width 1
 * up to s = 64, then panels growing by 10 % per step; the integrand is
 * analytic, so each panel is exact to rounding. */
static double vandriest_f(double s, double kappa, double Ap) {
  double m = 2.0 * kappa * s * (1.0 - exp(-s / Ap));
  return 2.0 / (1.0 + sqrt(1.0 + m * m));
}

int orc_vandriest(double yp, double kappa, double Ap, double *U_out, double *dU_out) {
  if (!(yp >= 0.0) || !(kappa > 0.0) || !(Ap > 0.0)) return -1;
  double x[ORC_MAXN], w[ORC_MAXN];
  orc_gauss(12, x, w);
  double U = 0.0, a = 0.0;
  while (a < yp) {
    double width = a < 64.0 ? 1.0 : 0.1 * a;
    double b = a + width < yp ? a + width : yp;
    double sum = 0.0;
    for (int q = 0; q < 12; ++q) sum += w[q] * vandriest_f(a + (b - a) * x[q], kappa, Ap);
    U += (b - a) * sum;
    a = b;
  }
  *U_out = U;
  *dU_out = vandriest_f(yp, kappa, Ap);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Mesh and geometry                                                          */
/* ------------------------------------------------------------------------ */

typedef struct {
  orc_params P;
  int64_t ncell;
  double *eta;        /* ny+1 wall-normal vertex parameters (tanh graded) */
  int64_t *enr;       /* enriched index per cell, -1 if not enriched */
  int64_t nenr;
  int npu, npp;       /* nodes per direction: k_u+1, k_p+1 */
  double glu[ORC_MAXN], glp[ORC_MAXN];
  double qu[ORC_MAXN], wu[ORC_MAXN];
  double qwn[ORC_MAXN], wwn[ORC_MAXN];
  double qp[ORC_MAXN], wp[ORC_MAXN];
  const double *tau;  /* wall shear stress per wall-face quadrature point */
  const double *tau_nodes; /* or: nodal wall shear stress [wall][nz][nx] (Sec. 3.2, m = 1) */
  signed char *act;   /* per enriched cell: 1 enrichment on, 0 off; NULL: all on */
  int conv_only;      /* velocity residual: 1 keeps the convective terms alone */
  int nle;            /* enrichment shape functions per component: (l+1)^3 = 1 or 8 */
} ctx;

/* Wall-normal vertex coordinate, Sec. 5.1: f(t) = tanh(gamma(2t-1))/tanh(gamma). */
void orc_vertex_eta(const orc_params *P, double *eta) {
  for (int j = 0; j <= P->ny; ++j) {
    double t = (double)j / P->ny;
    eta[j] = (P->gamma > 0) ? tanh(P->gamma * (2.0 * t - 1.0)) / tanh(P->gamma)
                            : 2.0 * t - 1.0;
  }
}

static double wall_lower_y(const ctx *C, double x) {
  return -1.0 + C->P.wall_amp * cos(2.0 * M_PI * x / C->P.Lx);
}

/* Analytic map of the channel (flat: y = eta; curved lower wall: the column
 * between y_w(x) and +1 is stretched linearly in eta). */
static double analytic_y(const ctx *C, double x, double eta) {
  double yw = wall_lower_y(C, x);
  return yw + 0.5 * (eta + 1.0) * (1.0 - yw);
}

static int is_curved(const ctx *C) { return C->P.wall_amp != 0.0; }

static void cell_index(const ctx *C, int64_t e, int *ex, int *ey, int *ez) {
  *ex = (int)(e % C->P.nx);
  *ey = (int)((e / C->P.nx) % C->P.ny);
  *ez = (int)(e / ((int64_t)C->P.nx * C->P.ny));
}

/* Map reference point xi in [0,1]^3 of cell e to physical X and Jacobian
 * J[d][a] = dX_d / dxi_a.  Flat walls: affine.  Curved wall: isoparametric of
 * degree k_u through the analytic map sampled at the cell's Gauss-Lobatto
 * points (only y is non-affine). */
static void cell_map(const ctx *C, int64_t e, const double xi[3], double X[3], double J[3][3]) {
  int ex, ey, ez;
  cell_index(C, e, &ex, &ey, &ez);
  double hx = C->P.Lx / C->P.nx, hz = C->P.Lz / C->P.nz;
  double x0 = ex * hx, z0 = ez * hz;
  double e0 = C->eta[ey], he = C->eta[ey + 1] - C->eta[ey];
  memset(J, 0, 9 * sizeof(double));
  X[0] = x0 + hx * xi[0];
  X[2] = z0 + hz * xi[2];
  J[0][0] = hx;
  J[2][2] = hz;
  if (!is_curved(C)) {
    X[1] = e0 + he * xi[1];
    J[1][1] = he;
    return;
  }
  int n = C->npu;
  double vx[ORC_MAXN], dx[ORC_MAXN], vy[ORC_MAXN], dy[ORC_MAXN];
  orc_lagrange(n, C->glu, xi[0], vx, dx);
  orc_lagrange(n, C->glu, xi[1], vy, dy);
  double y = 0, yx = 0, yy = 0;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      double Y = analytic_y(C, x0 + hx * C->glu[i], e0 + he * C->glu[j]);
      y += vx[i] * vy[j] * Y;
      yx += dx[i] * vy[j] * Y;
      yy += vx[i] * dy[j] * Y;
    }
  X[1] = y;
  J[1][0] = yx;
  J[1][1] = yy;
}

static double inv3(const double J[3][3], double Ji[3][3]) {
  double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
               J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
               J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
  Ji[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) / det;
  Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
  Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
  Ji[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) / det;
  Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
  Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
  Ji[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) / det;
  Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
  Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
  return det;
}

/* Geometry at the point xi of face (d, s) of cell e (xi[d] = s): physical
 * point X, inverse Jacobian Ji, outward unit normal nv and the area element
 * dA per unit reference-face area.  Nanson's relation for the map x(xi):
 * n dA = det(J) J^{-T} N dA_ref with the reference normal N = -e_d (s = 0) or
 * +e_d (s = 1); the d-th column of J^{-T} is the d-th row of J^{-1}, so
 * nv = sg Ji[d][:] / |Ji[d][:]| and dA = |det J| |Ji[d][:]|. */
static void face_point(const ctx *C, int64_t e, int d, int s, const double xi[3], double X[3], double Ji[3][3],
                       double nv[3], double *dA) {
  double J[3][3];
  cell_map(C, e, xi, X, J);
  double det = fabs(inv3(J, Ji));
  double sg = s ? 1.0 : -1.0;
  for (int k = 0; k < 3; ++k) nv[k] = sg * Ji[d][k];
  double nr = sqrt(nv[0] * nv[0] + nv[1] * nv[1] + nv[2] * nv[2]);
  for (int k = 0; k < 3; ++k) nv[k] /= nr;
  *dA = det * nr;
}

static int cell_enriched(const ctx *C, int ey) {
  if (C->P.fully_periodic) return 0;
  return (ey == 0 && C->P.enrich_lower) || (ey == C->P.ny - 1 && C->P.enrich_upper);
}

/* Number of Gauss points of the velocity rule in direction a for cell e. */
static int vel_nq(const ctx *C, int64_t e, int a) {
  int ex, ey, ez;
  cell_index(C, e, &ex, &ey, &ez);
  if (a == 1 && C->enr[e] >= 0) return C->P.nq_wn;
  return C->P.nq_u;
}

static const double *vel_q(const ctx *C, int64_t e, int a, const double **w) {
  if (a == 1 && C->enr[e] >= 0) { *w = C->wwn; return C->qwn; }
  *w = C->wu;
  return C->qu;
}

/* Face neighbour of cell e across face (d,s): returns -1 for a no-slip wall. */
static int64_t face_neighbor(const ctx *C, int64_t e, int d, int s) {
  int i[3];
  cell_index(C, e, &i[0], &i[1], &i[2]);
  int n[3] = {C->P.nx, C->P.ny, C->P.nz};
  int j = i[d] + (s ? 1 : -1);
  if (j < 0 || j >= n[d]) {
    if (d == 1 && !C->P.fully_periodic) return -1;
    j = (j + n[d]) % n[d];
  }
  i[d] = j;
  return i[0] + (int64_t)C->P.nx * (i[1] + (int64_t)C->P.ny * i[2]);
}

/* |Omega_e| with the cell's own velocity (or pressure) rule. */
static double cell_volume(const ctx *C, int64_t e, int pressure) {
  const double *q[3], *w[3];
  int n[3];
  for (int a = 0; a < 3; ++a) {
    if (pressure) { q[a] = C->qp; w[a] = C->wp; n[a] = C->P.nq_p; }
    else { q[a] = vel_q(C, e, a, &w[a]); n[a] = vel_nq(C, e, a); }
  }
  double vol = 0;
  for (int c = 0; c < n[2]; ++c)
    for (int b = 0; b < n[1]; ++b)
      for (int a = 0; a < n[0]; ++a) {
        double xi[3] = {q[0][a], q[1][b], q[2][c]}, X[3], J[3][3], Ji[3][3];
        cell_map(C, e, xi, X, J);
        vol += fabs(inv3(J, Ji)) * w[0][a] * w[1][b] * w[2][c];
      }
  return vol;
}

/* ------------------------------------------------------------------------ */
/* Wall distance y_h and the enrichment function psi (Sec. 3.2)              */
/* ------------------------------------------------------------------------ */

/* Distance of mesh vertex (ix, iy) to the closest wall node of wall w
 * (w = 0 lower, 1 upper).  Wall nodes of the linear wall mesh are the cell
 * vertices on the wall; rows are identical in z, so only x matters. */
static double vertex_wall_distance(const ctx *C, int ix, int iy, int w) {
  double hx = C->P.Lx / C->P.nx;
  double x = ix * hx, y = analytic_y(C, x, C->eta[iy]);
  if (w == 1) return fabs(1.0 - y);
  double best = INFINITY;
  for (int jx = 0; jx < C->P.nx; ++jx)
    for (int img = -1; img <= 1; ++img) {
      double xw = jx * hx + img * C->P.Lx;
      double dx = x - xw, dy = y - wall_lower_y(C, jx * hx);
      double d = sqrt(dx * dx + dy * dy);
      if (d < best) best = d;
    }
  return best;
}

typedef struct { double psi, g[3]; } psi_pt;

/* Wall distance and wall shear stress at reference point xi of enriched cell
 * e (Sec. 3.2), with their physical gradients (J^{-T} applied).
 * y_h: trilinear (m = 1) interpolation of the vertex wall distances.
 * tau_w: either the value of the wall-face Gauss column nearest to
 * (xi_x, xi_z) in the cell's velocity rule, treated as locally constant
 * (zero gradient), or, with nodal values, the bilinear interpolation
 * tau_w,h = sum_B N_B tau_w,B of the wall vertices, constant along the wall
 * normal (flat walls: x and z are affine in xi_x and xi_z). */
static void wall_fields(const ctx *C, int64_t e, const double xi[3], const double Ji[3][3], double *yh_out,
                        double gyh[3], double *tw_out, double gtw[3]) {
  int ex, ey, ez;
  cell_index(C, e, &ex, &ey, &ez);
  int w = (ey == 0) ? 0 : 1;
  double dv[2][2][2];
  for (int c = 0; c < 2; ++c)
    for (int b = 0; b < 2; ++b)
      for (int a = 0; a < 2; ++a)
        dv[c][b][a] = vertex_wall_distance(C, ex + a, ey + b, w);
  double yh = 0, gr[3] = {0, 0, 0};
  for (int c = 0; c < 2; ++c)
    for (int b = 0; b < 2; ++b)
      for (int a = 0; a < 2; ++a) {
        double lx = a ? xi[0] : 1 - xi[0], ly = b ? xi[1] : 1 - xi[1], lz = c ? xi[2] : 1 - xi[2];
        double sx = a ? 1 : -1, sy = b ? 1 : -1, sz = c ? 1 : -1;
        yh += dv[c][b][a] * lx * ly * lz;
        gr[0] += dv[c][b][a] * sx * ly * lz;
        gr[1] += dv[c][b][a] * lx * sy * lz;
        gr[2] += dv[c][b][a] * lx * ly * sz;
      }
  for (int d = 0; d < 3; ++d) gyh[d] = gr[0] * Ji[0][d] + gr[1] * Ji[1][d] + gr[2] * Ji[2][d];
  double tw = 0;
  gtw[0] = gtw[1] = gtw[2] = 0;
  if (C->tau_nodes) {
    double hx = C->P.Lx / C->P.nx, hz = C->P.Lz / C->P.nz;
    for (int c = 0; c < 2; ++c)
      for (int a = 0; a < 2; ++a) {
        int jx = (ex + a) % C->P.nx, jz = (ez + c) % C->P.nz;
        double tb = C->tau_nodes[((int64_t)w * C->P.nz + jz) * C->P.nx + jx];
        double nxa = a ? xi[0] : 1 - xi[0], nzc = c ? xi[2] : 1 - xi[2];
        tw += nxa * nzc * tb;
        gtw[0] += (a ? 1.0 : -1.0) / hx * nzc * tb;
        gtw[2] += nxa * (c ? 1.0 : -1.0) / hz * tb;
      }
  } else {
    /* nearest Gauss column of the velocity rule */
    int nq = C->P.nq_u, qx = 0, qz = 0;
    for (int q = 1; q < nq; ++q) {
      if (fabs(xi[0] - C->qu[q]) < fabs(xi[0] - C->qu[qx])) qx = q;
      if (fabs(xi[2] - C->qu[q]) < fabs(xi[2] - C->qu[qz])) qz = q;
    }
    int64_t ti = (((int64_t)w * C->P.nz + ez) * C->P.nx + ex) * nq * nq + (int64_t)qz * nq + qx;
    tw = C->tau[ti];
  }
  *yh_out = yh;
  *tw_out = tw;
}

/* psi and grad(psi) at reference point xi of enriched cell e:
 * y+ = y_h sqrt(tau_w)/nu (rho = 1), psi = U(y+) of the chosen law and
 * grad psi = U'(y+) grad y+ with
 * grad y+ = sqrt(tau_w)/nu grad y_h + y_h / (2 nu sqrt(tau_w)) grad tau_w.
 * A cell whose enrichment is switched off has psi = 0. */
static void eval_psi(const ctx *C, int64_t e, const double xi[3], const double Ji[3][3], psi_pt *out) {
  if (C->act && !C->act[C->enr[e]]) {
    out->psi = 0;
    out->g[0] = out->g[1] = out->g[2] = 0;
    return;
  }
  double yh, gyh[3], tw, gtw[3];
  wall_fields(C, e, xi, Ji, &yh, gyh, &tw, gtw);
  double st = sqrt(tw) / C->P.nu;
  double U, dU;
  if (C->P.psi_kind == 1)
    orc_vandriest(yh * st, C->P.kappa, C->P.A_plus, &U, &dU);
  else
    orc_spalding(yh * st, C->P.kappa, C->P.B, &U, &dU);
  out->psi = U;
  for (int d = 0; d < 3; ++d) out->g[d] = dU * (st * gyh[d] + yh / (2.0 * C->P.nu * sqrt(tw)) * gtw[d]);
}

/* Switch-off rule of Sec. 3.2: the enrichment of a wall cell is on when at
 * least one quadrature point of the cell (its enriched volume rule) has
 * y+ >= yplus_off.  Sets C->act (all on when yplus_off <= 0). */
static int cell_on(const ctx *C, int64_t e) {
  const double *q[3], *w[3];
  int nq[3];
  for (int a = 0; a < 3; ++a) { q[a] = vel_q(C, e, a, &w[a]); nq[a] = vel_nq(C, e, a); }
  for (int c = 0; c < nq[2]; ++c)
    for (int b = 0; b < nq[1]; ++b)
      for (int a = 0; a < nq[0]; ++a) {
        double xi[3] = {q[0][a], q[1][b], q[2][c]}, X[3], J[3][3], Ji[3][3], yh, gyh[3], tw, gtw[3];
        cell_map(C, e, xi, X, J);
        inv3(J, Ji);
        wall_fields(C, e, xi, Ji, &yh, gyh, &tw, gtw);
        if (yh * sqrt(tw) / C->P.nu >= C->P.yplus_off) return 1;
      }
  return 0;
}

/* Activity of every enriched cell (only `one` when one >= 0). */
static void ctx_activity(ctx *C, int64_t one) {
  if (!(C->P.yplus_off > 0) || C->nenr == 0) return;
  C->act = (signed char *)malloc((size_t)C->nenr);
  for (int64_t e = 0; e < C->ncell; ++e)
    if (C->enr[e] >= 0 && (one < 0 || e == one)) C->act[C->enr[e]] = (signed char)cell_on(C, e);
}

/* ------------------------------------------------------------------------ */
/* Point evaluation                                                          */
/* ------------------------------------------------------------------------ */

#define NP3MAX (ORC_MAXN * ORC_MAXN * ORC_MAXN)

typedef struct {
  double u[3], g[3][3];   /* velocity and g[c][d] = d u_c / d x_d */
  psi_pt psi;             /* valid if enriched */
  int enriched;
  /* valid if enriched: the enrichment functions psi N^l_B (B < (l+1)^3) and
   * their physical gradients N^l_B grad psi + psi grad N^l_B */
  double ev[8], eg[8][3];
} vel_pt;

/* Tensor-product basis of degree n-1 at xi, physical gradients via J^{-T}. */
static void basis3(int n, const double *nodes, const double xi[3], const double Ji[3][3],
                   double *bv, double (*bg)[3]) {
  double v[3][ORC_MAXN], d[3][ORC_MAXN];
  for (int a = 0; a < 3; ++a) orc_lagrange(n, nodes, xi[a], v[a], d[a]);
  for (int m = 0; m < n; ++m)
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < n; ++i) {
        int B = i + n * (j + n * m);
        double gx = d[0][i] * v[1][j] * v[2][m];
        double gy = v[0][i] * d[1][j] * v[2][m];
        double gz = v[0][i] * v[1][j] * d[2][m];
        bv[B] = v[0][i] * v[1][j] * v[2][m];
        for (int dd = 0; dd < 3; ++dd) bg[B][dd] = gx * Ji[0][dd] + gy * Ji[1][dd] + gz * Ji[2][dd];
      }
}

/* Enrichment functions of an enriched cell at xi (Sec. 3.1, eq.
 * enrichment): psi N^l_B with N^l_B the tensor-product Lagrange functions of
 * degree l on the nodes {0, 1} (l = 1: the trilinear vertex functions,
 * B = bx + 2 (by + 2 bz); l = 0: the constant 1), and their gradients. */
static void enr_basis(const ctx *C, const double xi[3], const double Ji[3][3], const psi_pt *ps, double *ev,
                      double (*eg)[3]) {
  if (C->nle == 1) {
    ev[0] = ps->psi;
    for (int d = 0; d < 3; ++d) eg[0][d] = ps->g[d];
    return;
  }
  static const double v01[2] = {0.0, 1.0};
  double nb[8], ng[8][3];
  basis3(2, v01, xi, Ji, nb, ng);
  for (int B = 0; B < 8; ++B) {
    ev[B] = ps->psi * nb[B];
    for (int d = 0; d < 3; ++d) eg[B][d] = nb[B] * ps->g[d] + ps->psi * ng[B][d];
  }
}

/* u_h = sum_B N_B u_B + psi sum_B N^l_B u~_B and its gradient at xi of cell e.
 * absmode: every product and sum taken in absolute value (rounding bounds). */
static void eval_vel(const ctx *C, const double *u, int64_t e, const double xi[3], const double Ji[3][3],
                     int absmode, vel_pt *out, double *bv, double (*bg)[3]) {
  int n = C->npu, np3 = n * n * n;
  basis3(n, C->glu, xi, Ji, bv, bg);
  for (int c = 0; c < 3; ++c) {
    const double *uc = u + ((int64_t)e * 3 + c) * np3;
    double s = 0, g0 = 0, g1 = 0, g2 = 0;
    for (int B = 0; B < np3; ++B) {
      double ub = absmode ? fabs(uc[B]) : uc[B];
      double b0 = absmode ? fabs(bv[B]) : bv[B];
      s += b0 * ub;
      g0 += (absmode ? fabs(bg[B][0]) : bg[B][0]) * ub;
      g1 += (absmode ? fabs(bg[B][1]) : bg[B][1]) * ub;
      g2 += (absmode ? fabs(bg[B][2]) : bg[B][2]) * ub;
    }
    out->u[c] = s;
    out->g[c][0] = g0; out->g[c][1] = g1; out->g[c][2] = g2;
  }
  out->enriched = (C->enr[e] >= 0);
  if (out->enriched) {
    eval_psi(C, e, xi, Ji, &out->psi);
    enr_basis(C, xi, Ji, &out->psi, out->ev, out->eg);
    const int nle = C->nle;
    const double *ut = u + C->ncell * 3 * np3 + C->enr[e] * 3 * nle;  /* [c][B] */
    for (int c = 0; c < 3; ++c)
      for (int B = 0; B < nle; ++B) {
        double uc = absmode ? fabs(ut[c * nle + B]) : ut[c * nle + B];
        double ps = absmode ? fabs(out->ev[B]) : out->ev[B];
        out->u[c] += ps * uc;
        for (int d = 0; d < 3; ++d) out->g[c][d] += uc * (absmode ? fabs(out->eg[B][d]) : out->eg[B][d]);
      }
  }
}

/* ------------------------------------------------------------------------ */
/* Context                                                                   */
/* ------------------------------------------------------------------------ */

static int ctx_init(ctx *C, const orc_params *P, const double *tau) {
  /* (tau_nodes is set by the callers that take nodal values) */
  memset(C, 0, sizeof(*C));
  C->P = *P;
  if (P->nx < 1 || P->ny < 1 || P->nz < 1) return -1;
  if (P->k_u < 1 || P->k_u + 1 > ORC_MAXN || P->k_p < 1 || P->k_p + 1 > ORC_MAXN) return -1;
  if (P->nq_u < 1 || P->nq_u > ORC_MAXN || P->nq_wn < 1 || P->nq_wn > ORC_MAXN ||
      P->nq_p < 1 || P->nq_p > ORC_MAXN) return -1;
  if (P->enrich_degree != 0 && P->enrich_degree != 1) return -1;
  C->nle = P->enrich_degree ? 8 : 1;
  C->ncell = (int64_t)P->nx * P->ny * P->nz;
  C->eta = (double *)malloc(sizeof(double) * (P->ny + 1));
  C->enr = (int64_t *)malloc(sizeof(int64_t) * C->ncell);
  orc_vertex_eta(P, C->eta);
  C->nenr = 0;
  for (int64_t e = 0; e < C->ncell; ++e) {
    int ex, ey, ez;
    cell_index(C, e, &ex, &ey, &ez);
    C->enr[e] = cell_enriched(C, ey) ? C->nenr++ : -1;
  }
  C->npu = P->k_u + 1;
  C->npp = P->k_p + 1;
  orc_gauss_lobatto(C->npu, C->glu);
  orc_gauss_lobatto(C->npp, C->glp);
  orc_gauss(P->nq_u, C->qu, C->wu);
  orc_gauss(P->nq_wn, C->qwn, C->wwn);
  orc_gauss(P->nq_p, C->qp, C->wp);
  C->tau = tau;
  return 0;
}

static void ctx_free(ctx *C) {
  free(C->eta);
  free(C->enr);
  free(C->act);
}

/* Operators built for constant enrichment weights (l = 0) only. */
static int ctx_init_l0(ctx *C, const orc_params *P, const double *tau) {
  if (ctx_init(C, P, tau)) return -1;
  if (C->nle != 1) { ctx_free(C); return -1; }
  return 0;
}

int64_t orc_num_dofs(const orc_params *P, int field) {
  ctx C;
  if (ctx_init(&C, P, NULL)) return -1;
  int64_t n;
  if (field == 0) n = C.ncell * 3 * C.npu * C.npu * C.npu + C.nenr * 3 * C.nle;
  else n = C.ncell * C.npp * C.npp * C.npp;
  ctx_free(&C);
  return n;
}

int64_t orc_num_enriched(const orc_params *P) {
  ctx C;
  if (ctx_init(&C, P, NULL)) return -1;
  int64_t n = C.nenr;
  ctx_free(&C);
  return n;
}

/* ------------------------------------------------------------------------ */
/* Velocity residual                                                         */
/* ------------------------------------------------------------------------ */

/* Residual of cell e for every test function of e (polynomial N_B e_c and,
 * if enriched, psi N^l_B e_c):
 *   r(phi) = (grad phi, 2 nu eps(u) - u (x) u)_e
 *          + sum_F ( phi . f_v + grad phi : F_g )_F
 *   f_v = 1/2 (u- (u-.n) + u+ (u+.n)) + Lambda/2 (u- - u+)
 *         - 1/2 (2nu eps(u-) + 2nu eps(u+)) n + tau_F nu (u- - u+)
 *   F_g = -theta nu sym((u- - u+) (x) n),   Lambda = max(2|u-.n|, 2|u+.n|)
 * so that M du/dt = -r (convective minus viscous weak forms of Sec. 4.2).
 * No-slip wall: u+ = -u-, grad u+ = grad u-, tau_F multiplied by
 * wall_ip_mult. */
static void vel_cell(const ctx *C, const double *u, int64_t e, double *r, int absmode,
                     double *bv, double (*bg)[3], double *bv2, double (*bg2)[3]) {
  int n = C->npu, np3 = n * n * n;
  /* every viscous term carries nu; the convective form F^c drops them (psi
   * keeps the physical nu through y+) */
  double nu = C->conv_only ? 0.0 : C->P.nu, theta = C->P.theta;
  double *re = r + (int64_t)e * 3 * np3;
  const int nle = C->nle;
  double rt[3 * 8] = {0};  /* enrichment rows [c][B] */
  for (int i = 0; i < 3 * np3; ++i) re[i] = 0.0;

  /* volume */
  {
    const double *q[3], *w[3];
    int nq[3];
    for (int a = 0; a < 3; ++a) { q[a] = vel_q(C, e, a, &w[a]); nq[a] = vel_nq(C, e, a); }
    for (int c3 = 0; c3 < nq[2]; ++c3)
      for (int b = 0; b < nq[1]; ++b)
        for (int a = 0; a < nq[0]; ++a) {
          double xi[3] = {q[0][a], q[1][b], q[2][c3]}, X[3], J[3][3], Ji[3][3];
          cell_map(C, e, xi, X, J);
          double wq = fabs(inv3(J, Ji)) * w[0][a] * w[1][b] * w[2][c3];
          vel_pt p;
          eval_vel(C, u, e, xi, Ji, absmode, &p, bv, bg);
          double G[3][3];
          for (int c = 0; c < 3; ++c)
            for (int d = 0; d < 3; ++d)
              G[c][d] = absmode ? nu * (p.g[c][d] + p.g[d][c]) + p.u[c] * p.u[d]
                                : nu * (p.g[c][d] + p.g[d][c]) - p.u[c] * p.u[d];
          for (int c = 0; c < 3; ++c) {
            double *rc = re + c * np3;
            for (int B = 0; B < np3; ++B) {
              double s = 0;
              for (int d = 0; d < 3; ++d) s += (absmode ? fabs(bg[B][d]) : bg[B][d]) * G[c][d];
              rc[B] += wq * s;
            }
            if (p.enriched)
              for (int B = 0; B < nle; ++B)
                for (int d = 0; d < 3; ++d) rt[c * nle + B] += wq * (absmode ? fabs(p.eg[B][d]) : p.eg[B][d]) * G[c][d];
          }
        }
  }

  /* faces */
  double vol_e = cell_volume(C, e, 0);
  for (int f = 0; f < 6; ++f) {
    int d = f / 2, s = f % 2;
    int t1 = (d == 0) ? 1 : 0, t2 = (d == 2) ? 1 : 2;
    int64_t nb = face_neighbor(C, e, d, s);
    int wall = (nb < 0);
    /* tangential rules: the larger count of the two adjacent cells */
    const double *q1, *w1, *q2, *w2;
    int n1 = vel_nq(C, e, t1), n2 = vel_nq(C, e, t2);
    q1 = vel_q(C, e, t1, &w1);
    q2 = vel_q(C, e, t2, &w2);
    if (!wall) {
      if (vel_nq(C, nb, t1) > n1) { n1 = vel_nq(C, nb, t1); q1 = vel_q(C, nb, t1, &w1); }
      if (vel_nq(C, nb, t2) > n2) { n2 = vel_nq(C, nb, t2); q2 = vel_q(C, nb, t2, &w2); }
    }
    /* face area with the face rule on e */
    double area = 0;
    for (int b = 0; b < n2; ++b)
      for (int a = 0; a < n1; ++a) {
        double xi[3], X[3], Ji[3][3], nv[3], dA;
        xi[d] = s; xi[t1] = q1[a]; xi[t2] = q2[b];
        face_point(C, e, d, s, xi, X, Ji, nv, &dA);
        area += dA * w1[a] * w2[b];
      }
    double pf = C->P.ip_factor_u * (double)(n) * (double)(n);
    double tauF;
    if (wall) tauF = C->P.wall_ip_mult * pf * area / vol_e;
    else tauF = pf * fmax(area / vol_e, area / cell_volume(C, nb, 0));

    for (int b = 0; b < n2; ++b)
      for (int a = 0; a < n1; ++a) {
        double xi[3], xn[3], X[3], Ji[3][3], Xn[3], Jn[3][3], Jin[3][3], nv[3], dA;
        xi[d] = s; xi[t1] = q1[a]; xi[t2] = q2[b];
        face_point(C, e, d, s, xi, X, Ji, nv, &dA);
        double wf = dA * w1[a] * w2[b];
        vel_pt pm, pp;
        eval_vel(C, u, e, xi, Ji, absmode, &pm, bv, bg);
        if (wall) {
          for (int c = 0; c < 3; ++c) {
            pp.u[c] = absmode ? pm.u[c] : -pm.u[c];
            for (int k = 0; k < 3; ++k) pp.g[c][k] = pm.g[c][k];
          }
        } else {
          xn[d] = 1 - s; xn[t1] = xi[t1]; xn[t2] = xi[t2];
          cell_map(C, nb, xn, Xn, Jn);
          inv3(Jn, Jin);
          eval_vel(C, u, nb, xn, Jin, absmode, &pp, bv2, bg2);
        }
        double fv[3], Fg[3][3];
        if (!absmode) {
          double unm = 0, unp = 0;
          for (int k = 0; k < 3; ++k) { unm += pm.u[k] * nv[k]; unp += pp.u[k] * nv[k]; }
          double lam = fmax(2.0 * fabs(unm), 2.0 * fabs(unp));
          double jmp[3];
          for (int c = 0; c < 3; ++c) jmp[c] = pm.u[c] - pp.u[c];
          for (int c = 0; c < 3; ++c) {
            double visc = 0;
            for (int k = 0; k < 3; ++k)
              visc += (pm.g[c][k] + pm.g[k][c] + pp.g[c][k] + pp.g[k][c]) * nv[k];
            fv[c] = 0.5 * (pm.u[c] * unm + pp.u[c] * unp) + 0.5 * lam * jmp[c] - 0.5 * nu * visc +
                    tauF * nu * jmp[c];
            for (int k = 0; k < 3; ++k) Fg[c][k] = -theta * nu * 0.5 * (jmp[c] * nv[k] + jmp[k] * nv[c]);
          }
        } else {
          double unm = 0, unp = 0, an[3];
          for (int k = 0; k < 3; ++k) an[k] = fabs(nv[k]);
          for (int k = 0; k < 3; ++k) { unm += pm.u[k] * an[k]; unp += pp.u[k] * an[k]; }
          double lam = 2.0 * fmax(unm, unp);
          double jmp[3];
          for (int c = 0; c < 3; ++c) jmp[c] = pm.u[c] + pp.u[c];
          for (int c = 0; c < 3; ++c) {
            double visc = 0;
            for (int k = 0; k < 3; ++k)
              visc += (pm.g[c][k] + pm.g[k][c] + pp.g[c][k] + pp.g[k][c]) * an[k];
            fv[c] = 0.5 * (pm.u[c] * unm + pp.u[c] * unp) + 0.5 * lam * jmp[c] + 0.5 * nu * visc +
                    tauF * nu * jmp[c];
            for (int k = 0; k < 3; ++k) Fg[c][k] = fabs(theta) * nu * 0.5 * (jmp[c] * an[k] + jmp[k] * an[c]);
          }
        }
        for (int c = 0; c < 3; ++c) {
          double *rc = re + c * np3;
          for (int B = 0; B < np3; ++B) {
            double sv = (absmode ? fabs(bv[B]) : bv[B]) * fv[c];
            for (int k = 0; k < 3; ++k) sv += (absmode ? fabs(bg[B][k]) : bg[B][k]) * Fg[c][k];
            rc[B] += wf * sv;
          }
          if (pm.enriched)
            for (int B = 0; B < nle; ++B) {
              double sv = (absmode ? fabs(pm.ev[B]) : pm.ev[B]) * fv[c];
              for (int k = 0; k < 3; ++k) sv += (absmode ? fabs(pm.eg[B][k]) : pm.eg[B][k]) * Fg[c][k];
              rt[c * nle + B] += wf * sv;
            }
        }
      }
  }
  if (C->enr[e] >= 0) {
    double *ro = r + C->ncell * 3 * np3 + C->enr[e] * 3 * nle;
    for (int i = 0; i < 3 * nle; ++i) ro[i] = rt[i];
  }
}

static int velocity_residual(const orc_params *P, const double *u, const double *tau_w, const double *tau_nodes,
                             const int64_t *cells, int64_t ncells, double *r, int absmode, int conv_only) {
  ctx C;
  if (ctx_init(&C, P, tau_w)) return -1;
  C.tau_nodes = tau_nodes;
  C.conv_only = conv_only;
  if (C.nenr > 0 && !tau_w && !tau_nodes) { ctx_free(&C); return -2; }
  ctx_activity(&C, -1);
  int n = C.npu, np3 = n * n * n;
  int err = 0;
#pragma omp parallel
  {
    double *bv = (double *)malloc(sizeof(double) * np3 * 2);
    double(*bg)[3] = (double(*)[3])malloc(sizeof(double) * 3 * np3 * 2);
#pragma omp for schedule(dynamic, 4)
    for (int64_t i = 0; i < ncells; ++i) {
      int64_t e = cells[i];
      if (e < 0 || e >= C.ncell) { err = -3; continue; }
      vel_cell(&C, u, e, r, absmode, bv, bg, bv + np3, bg + np3);
    }
    free(bv);
    free(bg);
  }
  ctx_free(&C);
  return err;
}

int orc_velocity_residual(const orc_params *P, const double *u, const double *tau_w,
                          const int64_t *cells, int64_t ncells, double *r, int absmode) {
  return velocity_residual(P, u, tau_w, NULL, cells, ncells, r, absmode, 0);
}

int orc_velocity_residual_nodal(const orc_params *P, const double *u, const double *tau_nodes,
                                const int64_t *cells, int64_t ncells, double *r, int absmode) {
  return velocity_residual(P, u, NULL, tau_nodes, cells, ncells, r, absmode, 0);
}

/* Convective form F^c_e of the explicit step (Sec. 4.1 eq. convstep, Sec. 4.2
 * eq. convstepspat): the residual's volume flux -u (x) u and face flux
 * {{u (x) u}} n + Lambda/2 (u- - u+), without the viscous terms. */
int orc_convective_residual(const orc_params *P, const double *u, const double *tau_w,
                            const int64_t *cells, int64_t ncells, double *r, int absmode) {
  return velocity_residual(P, u, tau_w, NULL, cells, ncells, r, absmode, 1);
}

/* ------------------------------------------------------------------------ */
/* Pressure gradient and velocity divergence terms (Sec. 4.2)                */
/* ------------------------------------------------------------------------ */

/* Face rule of face (d, s) of cell e: the tangential rules with the larger
 * point count of the two adjacent cells (as in the velocity residual). */
static void face_rule(const ctx *C, int64_t e, int64_t nb, int t1, int t2, const double **q1, const double **w1,
                      int *n1, const double **q2, const double **w2, int *n2) {
  *n1 = vel_nq(C, e, t1);
  *n2 = vel_nq(C, e, t2);
  *q1 = vel_q(C, e, t1, w1);
  *q2 = vel_q(C, e, t2, w2);
  if (nb >= 0) {
    if (vel_nq(C, nb, t1) > *n1) { *n1 = vel_nq(C, nb, t1); *q1 = vel_q(C, nb, t1, w1); }
    if (vel_nq(C, nb, t2) > *n2) { *n2 = vel_nq(C, nb, t2); *q2 = vel_q(C, nb, t2, w2); }
  }
}

/* pressure p_h = sum_B N^p_B p_B at xi of cell e */
static double eval_p(const ctx *C, const double *p, int64_t e, const double xi[3], const double Ji[3][3],
                     double *bv, double (*bg)[3]) {
  int n = C->npp, np3 = n * n * n;
  basis3(n, C->glp, xi, Ji, bv, bg);
  const double *pe = p + (int64_t)e * np3;
  double s = 0;
  for (int B = 0; B < np3; ++B) s += bv[B] * pe[B];
  return s;
}

/* Pressure gradient term for every velocity test function v of cell e
 * (N_B e_c and, in an enriched cell, the enrichment functions psi N^l_B e_c
 * of Sec. 3.1 eq. enrichment: psi e_c for l = 0):
 *   g(v) = -(div v, p)_e + (v . n, {{p}})_{boundary of e},  {{p}} = (p- + p+)/2,
 * with the external value p+ = p- on no-slip walls (the pressure's
 * homogeneous Neumann condition) and the velocity quadrature of the cell and
 * of its faces.  Out: velocity layout. */
static void grad_cell(const ctx *C, const double *p, int64_t e, double *g, double *bv, double (*bg)[3],
                      double *pv, double (*pg)[3]) {
  int n = C->npu, np3 = n * n * n;
  const int nle = C->nle;
  double *ge = g + (int64_t)e * 3 * np3;
  double gt[24] = {0};  /* [c][B] */
  double ev[8], eg[8][3];
  for (int i = 0; i < 3 * np3; ++i) ge[i] = 0.0;
  int enriched = C->enr[e] >= 0;
  const double *q[3], *w[3];
  int nq[3];
  for (int a = 0; a < 3; ++a) { q[a] = vel_q(C, e, a, &w[a]); nq[a] = vel_nq(C, e, a); }
  for (int c3 = 0; c3 < nq[2]; ++c3)
    for (int b = 0; b < nq[1]; ++b)
      for (int a = 0; a < nq[0]; ++a) {
        double xi[3] = {q[0][a], q[1][b], q[2][c3]}, X[3], J[3][3], Ji[3][3];
        cell_map(C, e, xi, X, J);
        double wq = fabs(inv3(J, Ji)) * w[0][a] * w[1][b] * w[2][c3];
        double ph = eval_p(C, p, e, xi, Ji, pv, pg);
        basis3(n, C->glu, xi, Ji, bv, bg);
        /* div (N_B e_c) = d_c N_B */
        for (int c = 0; c < 3; ++c)
          for (int B = 0; B < np3; ++B) ge[c * np3 + B] -= wq * bg[B][c] * ph;
        if (enriched) {
          psi_pt ps;
          eval_psi(C, e, xi, Ji, &ps);
          enr_basis(C, xi, Ji, &ps, ev, eg);
          /* div (psi N_B e_c) = d_c (psi N_B) */
          for (int c = 0; c < 3; ++c)
            for (int B = 0; B < nle; ++B) gt[c * nle + B] -= wq * eg[B][c] * ph;
        }
      }
  for (int f = 0; f < 6; ++f) {
    int d = f / 2, s = f % 2;
    int t1 = (d == 0) ? 1 : 0, t2 = (d == 2) ? 1 : 2;
    int64_t nb = face_neighbor(C, e, d, s);
    const double *q1, *w1, *q2, *w2;
    int n1, n2;
    face_rule(C, e, nb, t1, t2, &q1, &w1, &n1, &q2, &w2, &n2);
    for (int b = 0; b < n2; ++b)
      for (int a = 0; a < n1; ++a) {
        double xi[3], X[3], Ji[3][3], nv[3], dA;
        xi[d] = s; xi[t1] = q1[a]; xi[t2] = q2[b];
        face_point(C, e, d, s, xi, X, Ji, nv, &dA);
        double wf = dA * w1[a] * w2[b];
        double pm = eval_p(C, p, e, xi, Ji, pv, pg), pp = pm;
        if (nb >= 0) {
          double xn[3], Xn[3], Jn[3][3], Jin[3][3];
          xn[d] = 1 - s; xn[t1] = xi[t1]; xn[t2] = xi[t2];
          cell_map(C, nb, xn, Xn, Jn);
          inv3(Jn, Jin);
          pp = eval_p(C, p, nb, xn, Jin, pv, pg);
        }
        double pavg = 0.5 * (pm + pp);
        basis3(n, C->glu, xi, Ji, bv, bg);
        for (int c = 0; c < 3; ++c)
          for (int B = 0; B < np3; ++B) ge[c * np3 + B] += wf * bv[B] * nv[c] * pavg;
        if (enriched) {
          psi_pt ps;
          eval_psi(C, e, xi, Ji, &ps);
          enr_basis(C, xi, Ji, &ps, ev, eg);
          for (int c = 0; c < 3; ++c)
            for (int B = 0; B < nle; ++B) gt[c * nle + B] += wf * ev[B] * nv[c] * pavg;
        }
      }
  }
  if (enriched) {
    double *go = g + C->ncell * 3 * np3 + C->enr[e] * 3 * nle;
    for (int i = 0; i < 3 * nle; ++i) go[i] = gt[i];
  }
}

/* Velocity divergence term for every pressure test function q of cell e:
 *   c(q) = -(grad q, u)_e + (q, {{u}} . n)_{boundary of e},  {{u}} = (u- + u+)/2,
 * u the full (enriched) velocity; on no-slip walls the interior value
 * {{u}} = u- (the boundary condition Sec. 4.2 gives for this term of the
 * pressure Poisson equation), and the velocity quadrature of the cell and of
 * its faces.  Out: pressure layout. */
static void div_cell(const ctx *C, const double *u, int64_t e, double *out, double *bv, double (*bg)[3],
                     double *bv2, double (*bg2)[3], double *pv, double (*pg)[3]) {
  int np = C->npp, np3p = np * np * np;
  double *oe = out + (int64_t)e * np3p;
  for (int i = 0; i < np3p; ++i) oe[i] = 0.0;
  const double *q[3], *w[3];
  int nq[3];
  for (int a = 0; a < 3; ++a) { q[a] = vel_q(C, e, a, &w[a]); nq[a] = vel_nq(C, e, a); }
  for (int c3 = 0; c3 < nq[2]; ++c3)
    for (int b = 0; b < nq[1]; ++b)
      for (int a = 0; a < nq[0]; ++a) {
        double xi[3] = {q[0][a], q[1][b], q[2][c3]}, X[3], J[3][3], Ji[3][3];
        cell_map(C, e, xi, X, J);
        double wq = fabs(inv3(J, Ji)) * w[0][a] * w[1][b] * w[2][c3];
        vel_pt vp;
        eval_vel(C, u, e, xi, Ji, 0, &vp, bv, bg);
        basis3(np, C->glp, xi, Ji, pv, pg);
        for (int B = 0; B < np3p; ++B)
          oe[B] -= wq * (pg[B][0] * vp.u[0] + pg[B][1] * vp.u[1] + pg[B][2] * vp.u[2]);
      }
  for (int f = 0; f < 6; ++f) {
    int d = f / 2, s = f % 2;
    int t1 = (d == 0) ? 1 : 0, t2 = (d == 2) ? 1 : 2;
    int64_t nb = face_neighbor(C, e, d, s);
    const double *q1, *w1, *q2, *w2;
    int n1, n2;
    face_rule(C, e, nb, t1, t2, &q1, &w1, &n1, &q2, &w2, &n2);
    for (int b = 0; b < n2; ++b)
      for (int a = 0; a < n1; ++a) {
        double xi[3], xn[3], X[3], Ji[3][3], Xn[3], Jn[3][3], Jin[3][3], nv[3], dA;
        xi[d] = s; xi[t1] = q1[a]; xi[t2] = q2[b];
        face_point(C, e, d, s, xi, X, Ji, nv, &dA);
        double wf = dA * w1[a] * w2[b];
        vel_pt pm, pp;
        eval_vel(C, u, e, xi, Ji, 0, &pm, bv, bg);
        if (nb >= 0) {
          xn[d] = 1 - s; xn[t1] = xi[t1]; xn[t2] = xi[t2];
          cell_map(C, nb, xn, Xn, Jn);
          inv3(Jn, Jin);
          eval_vel(C, u, nb, xn, Jin, 0, &pp, bv2, bg2);
        } else {
          pp = pm; /* interior value on a no-slip wall */
        }
        double un = 0;
        for (int k = 0; k < 3; ++k) un += 0.5 * (pm.u[k] + pp.u[k]) * nv[k];
        basis3(np, C->glp, xi, Ji, pv, pg);
        for (int B = 0; B < np3p; ++B) oe[B] += wf * pv[B] * un;
      }
  }
}

static int mixed_op(const orc_params *P, const double *in, const double *tau_w, const double *tau_nodes,
                    const int64_t *cells, int64_t ncells, double *out, int divergence) {
  ctx C;
  if (ctx_init(&C, P, tau_w)) return -1;
  C.tau_nodes = tau_nodes;
  if (C.nenr > 0 && !tau_w && !tau_nodes) { ctx_free(&C); return -2; }
  ctx_activity(&C, -1);
  int n = C.npu, np3 = n * n * n, npp3 = C.npp * C.npp * C.npp;
  int err = 0;
#pragma omp parallel
  {
    double *bv = (double *)malloc(sizeof(double) * (2 * np3 + npp3));
    double(*bg)[3] = (double(*)[3])malloc(sizeof(double) * 3 * (2 * np3 + npp3));
#pragma omp for schedule(dynamic, 4)
    for (int64_t i = 0; i < ncells; ++i) {
      int64_t e = cells[i];
      if (e < 0 || e >= C.ncell) { err = -3; continue; }
      if (divergence)
        div_cell(&C, in, e, out, bv, bg, bv + np3, bg + np3, bv + 2 * np3, bg + 2 * np3);
      else
        grad_cell(&C, in, e, out, bv, bg, bv + 2 * np3, bg + 2 * np3);
    }
    free(bv);
    free(bg);
  }
  ctx_free(&C);
  return err;
}

/* Pressure gradient term g = P p (velocity layout) of the listed cells. */
int orc_pressure_gradient(const orc_params *P, const double *p, const double *tau_w, const double *tau_nodes,
                          const int64_t *cells, int64_t ncells, double *g) {
  return mixed_op(P, p, tau_w, tau_nodes, cells, ncells, g, 0);
}

/* Velocity divergence term c = C u (pressure layout) of the listed cells. */
int orc_velocity_divergence(const orc_params *P, const double *u, const double *tau_w, const double *tau_nodes,
                            const int64_t *cells, int64_t ncells, double *c) {
  return mixed_op(P, u, tau_w, tau_nodes, cells, ncells, c, 1);
}

/* ------------------------------------------------------------------------ */
/* Div-div penalty (Sec. 4.2, eq. div-div)                                   */
/* ------------------------------------------------------------------------ */

/* tau_D of each listed cell: ||u||_e h_e dt_over_cr, ||u||_e the volume
 * average of |u| over the cell (the full velocity, with the cell's velocity
 * rule) and h_e the cube root of the cell volume. */
int orc_divdiv_tau(const orc_params *P, const double *u, const double *tau_w, const double *tau_nodes,
                   double dt_over_cr, const int64_t *cells, int64_t ncells, double *tau_d) {
  ctx C;
  if (ctx_init(&C, P, tau_w)) return -1;
  C.tau_nodes = tau_nodes;
  if (C.nenr > 0 && !tau_w && !tau_nodes) { ctx_free(&C); return -2; }
  ctx_activity(&C, -1);
  int n = C.npu, np3 = n * n * n;
  int err = 0;
#pragma omp parallel
  {
    double *bv = (double *)malloc(sizeof(double) * np3);
    double(*bg)[3] = (double(*)[3])malloc(sizeof(double) * 3 * np3);
#pragma omp for schedule(dynamic, 4)
    for (int64_t i = 0; i < ncells; ++i) {
      int64_t e = cells[i];
      if (e < 0 || e >= C.ncell) { err = -3; continue; }
      const double *q[3], *w[3];
      int nq[3];
      for (int a = 0; a < 3; ++a) { q[a] = vel_q(&C, e, a, &w[a]); nq[a] = vel_nq(&C, e, a); }
      double vol = 0, mag = 0;
      for (int c3 = 0; c3 < nq[2]; ++c3)
        for (int b = 0; b < nq[1]; ++b)
          for (int a = 0; a < nq[0]; ++a) {
            double xi[3] = {q[0][a], q[1][b], q[2][c3]}, X[3], J[3][3], Ji[3][3];
            cell_map(&C, e, xi, X, J);
            double wq = fabs(inv3(J, Ji)) * w[0][a] * w[1][b] * w[2][c3];
            vel_pt vp;
            eval_vel(&C, u, e, xi, Ji, 0, &vp, bv, bg);
            vol += wq;
            mag += wq * sqrt(vp.u[0] * vp.u[0] + vp.u[1] * vp.u[1] + vp.u[2] * vp.u[2]);
          }
      tau_d[e] = mag / vol * cbrt(vol) * dt_over_cr;
    }
    free(bv);
    free(bg);
  }
  ctx_free(&C);
  return err;
}

/* Div-div penalty D(v, u) = (div v, tau_D div u)_e for every velocity test
 * function v of the listed cells (N_B e_c, and psi N^l_B e_c in enriched cells),
 * u the full velocity, tau_D per cell, the cell's velocity rule.  Out:
 * velocity layout. */
int orc_divdiv_apply(const orc_params *P, const double *u, const double *tau_w, const double *tau_nodes,
                     const double *tau_d, const int64_t *cells, int64_t ncells, double *out) {
  ctx C;
  if (ctx_init(&C, P, tau_w)) return -1;
  C.tau_nodes = tau_nodes;
  if (C.nenr > 0 && !tau_w && !tau_nodes) { ctx_free(&C); return -2; }
  ctx_activity(&C, -1);
  int n = C.npu, np3 = n * n * n;
  const int nle = C.nle;
  int err = 0;
#pragma omp parallel
  {
    double *bv = (double *)malloc(sizeof(double) * np3);
    double(*bg)[3] = (double(*)[3])malloc(sizeof(double) * 3 * np3);
#pragma omp for schedule(dynamic, 4)
    for (int64_t i = 0; i < ncells; ++i) {
      int64_t e = cells[i];
      if (e < 0 || e >= C.ncell) { err = -3; continue; }
      double *oe = out + e * 3 * np3, ot[24] = {0};
      for (int k = 0; k < 3 * np3; ++k) oe[k] = 0.0;
      const double *q[3], *w[3];
      int nq[3];
      for (int a = 0; a < 3; ++a) { q[a] = vel_q(&C, e, a, &w[a]); nq[a] = vel_nq(&C, e, a); }
      for (int c3 = 0; c3 < nq[2]; ++c3)
        for (int b = 0; b < nq[1]; ++b)
          for (int a = 0; a < nq[0]; ++a) {
            double xi[3] = {q[0][a], q[1][b], q[2][c3]}, X[3], J[3][3], Ji[3][3];
            cell_map(&C, e, xi, X, J);
            double wq = fabs(inv3(J, Ji)) * w[0][a] * w[1][b] * w[2][c3];
            vel_pt vp;
            eval_vel(&C, u, e, xi, Ji, 0, &vp, bv, bg);
            double f = wq * tau_d[e] * (vp.g[0][0] + vp.g[1][1] + vp.g[2][2]);
            /* div (N_B e_c) = d_c N_B;  div (psi N^l_B e_c) = d_c (psi N^l_B) */
            for (int c = 0; c < 3; ++c)
              for (int B = 0; B < np3; ++B) oe[c * np3 + B] += bg[B][c] * f;
            if (vp.enriched)
              for (int c = 0; c < 3; ++c)
                for (int B = 0; B < nle; ++B) ot[c * nle + B] += vp.eg[B][c] * f;
          }
      if (C.enr[e] >= 0) {
        double *oo = out + C.ncell * 3 * np3 + C.enr[e] * 3 * nle;
        for (int k = 0; k < 3 * nle; ++k) oo[k] = ot[k];
      }
    }
    free(bv);
    free(bg);
  }
  ctx_free(&C);
  return err;
}

/* ------------------------------------------------------------------------ */
/* SIP Poisson operator                                                      */
/* ------------------------------------------------------------------------ */

/* (A p)(q) for every basis function q of cell e, A = -L with L the pressure
 * Laplace form of Sec. 4.2 (eq. ipflux) and homogeneous Neumann data on walls:
 *   (grad q, grad p)_e + sum_{F not wall} [ -1/2 (grad q.n)(p- - p+)
 *                                           - q ({{grad p}}.n - tau_F (p- - p+)) ]_F */
static void poisson_cell(const ctx *C, const double *p, int64_t e, double *y, int absmode,
                         double *bv, double (*bg)[3], double *bv2, double (*bg2)[3]) {
  int n = C->npp, np3 = n * n * n, nq = C->P.nq_p;
  double *ye = y + (int64_t)e * np3;
  const double *pe = p + (int64_t)e * np3;
  for (int B = 0; B < np3; ++B) ye[B] = 0.0;
  for (int c3 = 0; c3 < nq; ++c3)
    for (int b = 0; b < nq; ++b)
      for (int a = 0; a < nq; ++a) {
        double xi[3] = {C->qp[a], C->qp[b], C->qp[c3]}, X[3], J[3][3], Ji[3][3];
        cell_map(C, e, xi, X, J);
        double wq = fabs(inv3(J, Ji)) * C->wp[a] * C->wp[b] * C->wp[c3];
        basis3(n, C->glp, xi, Ji, bv, bg);
        double g[3] = {0, 0, 0};
        for (int B = 0; B < np3; ++B)
          for (int k = 0; k < 3; ++k)
            g[k] += absmode ? fabs(bg[B][k] * pe[B]) : bg[B][k] * pe[B];
        for (int B = 0; B < np3; ++B) {
          double s = 0;
          for (int k = 0; k < 3; ++k) s += (absmode ? fabs(bg[B][k]) : bg[B][k]) * g[k];
          ye[B] += wq * s;
        }
      }
  double vol_e = cell_volume(C, e, 1);
  for (int f = 0; f < 6; ++f) {
    int d = f / 2, s = f % 2;
    int t1 = (d == 0) ? 1 : 0, t2 = (d == 2) ? 1 : 2;
    int64_t nb = face_neighbor(C, e, d, s);
    if (nb < 0) continue; /* homogeneous Neumann wall: no face terms */
    const double *pn = p + nb * np3;
    double area = 0;
    for (int b = 0; b < nq; ++b)
      for (int a = 0; a < nq; ++a) {
        double xi[3], X[3], Ji[3][3], nv[3], dA;
        xi[d] = s; xi[t1] = C->qp[a]; xi[t2] = C->qp[b];
        face_point(C, e, d, s, xi, X, Ji, nv, &dA);
        area += dA * C->wp[a] * C->wp[b];
      }
    double tauF = C->P.ip_factor_p * (double)n * n * fmax(area / vol_e, area / cell_volume(C, nb, 1));
    for (int b = 0; b < nq; ++b)
      for (int a = 0; a < nq; ++a) {
        double xi[3], xn[3], X[3], Ji[3][3], Jn[3][3], Jin[3][3], nv[3], dA;
        xi[d] = s; xi[t1] = C->qp[a]; xi[t2] = C->qp[b];
        face_point(C, e, d, s, xi, X, Ji, nv, &dA);
        double wf = dA * C->wp[a] * C->wp[b];
        xn[d] = 1 - s; xn[t1] = xi[t1]; xn[t2] = xi[t2];
        cell_map(C, nb, xn, X, Jn);
        inv3(Jn, Jin);
        basis3(n, C->glp, xi, Ji, bv, bg);
        basis3(n, C->glp, xn, Jin, bv2, bg2);
        double pm = 0, pp = 0, gm = 0, gp = 0;
        for (int B = 0; B < np3; ++B) {
          double gnm = bg[B][0] * nv[0] + bg[B][1] * nv[1] + bg[B][2] * nv[2];
          double gnp = bg2[B][0] * nv[0] + bg2[B][1] * nv[1] + bg2[B][2] * nv[2];
          if (absmode) {
            pm += fabs(bv[B] * pe[B]); pp += fabs(bv2[B] * pn[B]);
            gm += fabs(gnm * pe[B]); gp += fabs(gnp * pn[B]);
          } else {
            pm += bv[B] * pe[B]; pp += bv2[B] * pn[B];
            gm += gnm * pe[B]; gp += gnp * pn[B];
          }
        }
        double jmp = absmode ? pm + pp : pm - pp;
        double avg = 0.5 * (gm + gp);
        double fval = absmode ? avg + tauF * jmp : -avg + tauF * jmp; /* tested with q */
        double fgrd = absmode ? 0.5 * jmp : -0.5 * jmp;               /* tested with grad q . n */
        for (int B = 0; B < np3; ++B) {
          double gnm = bg[B][0] * nv[0] + bg[B][1] * nv[1] + bg[B][2] * nv[2];
          if (absmode) ye[B] += wf * (fabs(bv[B]) * fval + fabs(gnm) * fgrd);
          else ye[B] += wf * (bv[B] * fval + gnm * fgrd);
        }
      }
  }
}

int orc_poisson_apply(const orc_params *P, const double *p, const int64_t *cells, int64_t ncells,
                      double *y, int absmode) {
  ctx C;
  if (ctx_init(&C, P, NULL)) return -1;
  int n = C.npp, np3 = n * n * n;
  int err = 0;
#pragma omp parallel
  {
    double *bv = (double *)malloc(sizeof(double) * np3 * 2);
    double(*bg)[3] = (double(*)[3])malloc(sizeof(double) * 3 * np3 * 2);
#pragma omp for schedule(dynamic, 8)
    for (int64_t i = 0; i < ncells; ++i) {
      int64_t e = cells[i];
      if (e < 0 || e >= C.ncell) { err = -3; continue; }
      poisson_cell(&C, p, e, y, absmode, bv, bg, bv + np3, bg + np3);
    }
    free(bv);
    free(bg);
  }
  ctx_free(&C);
  return err;
}

/* Diagonal of A: diag_B = (A e_B)_B with e_B the unit vector of basis function
 * B of cell e, evaluated by the same cell routine on a vector that is zero
 * everywhere else. */
int orc_poisson_diag(const orc_params *P, const int64_t *cells, int64_t ncells, double *dg) {
  ctx C;
  if (ctx_init(&C, P, NULL)) return -1;
  int n = C.npp, np3 = n * n * n;
  int64_t N = C.ncell * np3;
  int err = 0;
#pragma omp parallel
  {
    double *bv = (double *)malloc(sizeof(double) * np3 * 2);
    double(*bg)[3] = (double(*)[3])malloc(sizeof(double) * 3 * np3 * 2);
    double *unit = (double *)calloc(N, sizeof(double));
    double *out = (double *)calloc(N, sizeof(double));
#pragma omp for schedule(dynamic, 8)
    for (int64_t i = 0; i < ncells; ++i) {
      int64_t e = cells[i];
      if (e < 0 || e >= C.ncell) { err = -3; continue; }
      for (int B = 0; B < np3; ++B) {
        unit[e * np3 + B] = 1.0;
        poisson_cell(&C, unit, e, out, 0, bv, bg, bv + np3, bg + np3);
        dg[e * np3 + B] = out[e * np3 + B];
        unit[e * np3 + B] = 0.0;
      }
    }
    free(bv);
    free(bg);
    free(unit);
    free(out);
  }
  ctx_free(&C);
  return err;
}

/* psi and grad psi at a reference point of an enriched cell (for tests). */
int orc_psi_point(const orc_params *P, const double *tau_w, int64_t e, const double *xi, double *out4) {
  ctx C;
  if (ctx_init(&C, P, tau_w)) return -1;
  if (e < 0 || e >= C.ncell || C.enr[e] < 0) { ctx_free(&C); return -2; }
  ctx_activity(&C, e);
  double X[3], J[3][3], Ji[3][3];
  cell_map(&C, e, xi, X, J);
  inv3(J, Ji);
  psi_pt pt;
  eval_psi(&C, e, xi, Ji, &pt);
  out4[0] = pt.psi;
  out4[1] = pt.g[0]; out4[2] = pt.g[1]; out4[3] = pt.g[2];
  ctx_free(&C);
  return 0;
}

/* psi and grad psi with a nodal wall shear stress field tau_nodes
 * [wall][nz][nx] (Sec. 3.2): tau_w,h bilinear between the wall vertices, grad
 * psi with the grad tau_w term of the chain rule. */
int orc_psi_point_nodal(const orc_params *P, const double *tau_nodes, int64_t e, const double *xi, double *out4) {
  ctx C;
  if (ctx_init(&C, P, NULL)) return -1;
  C.tau_nodes = tau_nodes;
  if (e < 0 || e >= C.ncell || C.enr[e] < 0) { ctx_free(&C); return -2; }
  ctx_activity(&C, e);
  double X[3], J[3][3], Ji[3][3];
  cell_map(&C, e, xi, X, J);
  inv3(J, Ji);
  psi_pt pt;
  eval_psi(&C, e, xi, Ji, &pt);
  out4[0] = pt.psi;
  out4[1] = pt.g[0]; out4[2] = pt.g[1]; out4[3] = pt.g[2];
  ctx_free(&C);
  return 0;
}

/* psi at the points of the enriched volume rule (nq_u x nq_wn x nq_u, x
 * fastest) of each listed enriched cell, from the per-point tau_w or, when
 * given, the nodal tau_nodes; out: [ncells][points]. */
static int psi_volume(const orc_params *P, const double *tau_w, const double *tau_nodes, const int64_t *cells,
                      int64_t ncells, double *out, int with_grad);

int orc_psi_volume(const orc_params *P, const double *tau_w, const double *tau_nodes, const int64_t *cells,
                   int64_t ncells, double *out) {
  return psi_volume(P, tau_w, tau_nodes, cells, ncells, out, 0);
}

/* The same with grad psi: out [ncells][points][psi, dpsi/dx, dpsi/dy, dpsi/dz]. */
int orc_psi_volume4(const orc_params *P, const double *tau_w, const double *tau_nodes, const int64_t *cells,
                    int64_t ncells, double *out) {
  return psi_volume(P, tau_w, tau_nodes, cells, ncells, out, 1);
}

static int psi_volume(const orc_params *P, const double *tau_w, const double *tau_nodes, const int64_t *cells,
                      int64_t ncells, double *out, int with_grad) {
  ctx C;
  if (ctx_init(&C, P, tau_w)) return -1;
  C.tau_nodes = tau_nodes;
  if (C.nenr > 0 && !tau_w && !tau_nodes) { ctx_free(&C); return -2; }
  int err = 0;
  for (int64_t i = 0; i < ncells; ++i)
    if (cells[i] < 0 || cells[i] >= C.ncell || C.enr[cells[i]] < 0) err = -3;
  if (err) { ctx_free(&C); return err; }
  ctx_activity(&C, -1);
  int nq = P->nq_u, nw = P->nq_wn, npts = nq * nw * nq;
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t i = 0; i < ncells; ++i) {
    int64_t e = cells[i];
    for (int c = 0; c < nq; ++c)
      for (int b = 0; b < nw; ++b)
        for (int a = 0; a < nq; ++a) {
          double xi[3] = {C.qu[a], C.qwn[b], C.qu[c]}, X[3], J[3][3], Ji[3][3];
          cell_map(&C, e, xi, X, J);
          inv3(J, Ji);
          psi_pt pt;
          eval_psi(&C, e, xi, Ji, &pt);
          const int64_t o = i * npts + a + nq * (b + nw * c);
          if (with_grad) {
            out[o * 4] = pt.psi;
            for (int d = 0; d < 3; ++d) out[o * 4 + 1 + d] = pt.g[d];
          } else {
            out[o] = pt.psi;
          }
        }
  }
  ctx_free(&C);
  return 0;
}

/* Enrichment on (1) or off (0) per enriched cell under the switch-off rule
 * of Sec. 3.2 (all 1 when yplus_off <= 0); out: nenr flags. */
int orc_enrichment_active(const orc_params *P, const double *tau_w, const double *tau_nodes, int32_t *out) {
  ctx C;
  if (ctx_init(&C, P, tau_w)) return -1;
  C.tau_nodes = tau_nodes;
  if (C.nenr > 0 && !tau_w && !tau_nodes) { ctx_free(&C); return -2; }
  ctx_activity(&C, -1);
  for (int64_t k = 0; k < C.nenr; ++k) out[k] = C.act ? C.act[k] : 1;
  ctx_free(&C);
  return 0;
}

/* Nodal wall shear stress of both walls (Sec. 3.2):
 *   tau_w,B = || int_{wall} N_B tau_w dA || / int_{wall} N_B dA,
 * tau_w = nu (grad u_h) n with the outward normal n = -e_y (lower wall) or
 * +e_y (upper wall) and u_h the full (enriched) velocity, whose psi comes
 * from the current tau field (tau_w per point, or tau_nodes when given);
 * N_B the bilinear hat function of wall vertex B, both integrals by the
 * velocity rule's Gauss points on the wall faces.  Flat walls only.
 * out: [wall][nz][nx]. */
int orc_wall_shear_nodes(const orc_params *P, const double *u, const double *tau_w, const double *tau_nodes,
                         double *out) {
  ctx C;
  if (P->fully_periodic || P->wall_amp != 0.0) return -3;
  if (ctx_init(&C, P, tau_w)) return -1;
  C.tau_nodes = tau_nodes;
  if (C.nenr > 0 && !tau_w && !tau_nodes) { ctx_free(&C); return -2; }
  ctx_activity(&C, -1);
  int nx = P->nx, nz = P->nz, nq = P->nq_u, n = C.npu, np3 = n * n * n;
  double hx = P->Lx / nx, hz = P->Lz / nz;
  double *num = (double *)calloc((size_t)2 * nz * nx * 3, sizeof(double));
  double *den = (double *)calloc((size_t)2 * nz * nx, sizeof(double));
  double *bv = (double *)malloc(sizeof(double) * np3 * 4);
  double(*bg)[3] = (double(*)[3])(bv + np3);
  for (int w = 0; w < 2; ++w) {
    int ey = w ? P->ny - 1 : 0;
    double ny_out = w ? 1.0 : -1.0;
    for (int ez = 0; ez < nz; ++ez)
      for (int ex = 0; ex < nx; ++ex) {
        int64_t e = ex + (int64_t)nx * (ey + (int64_t)P->ny * ez);
        for (int qz = 0; qz < nq; ++qz)
          for (int qx = 0; qx < nq; ++qx) {
            double xi[3] = {C.qu[qx], w ? 1.0 : 0.0, C.qu[qz]};
            double X[3], J[3][3], Ji[3][3];
            cell_map(&C, e, xi, X, J);
            inv3(J, Ji);
            vel_pt vp;
            eval_vel(&C, u, e, xi, Ji, 0, &vp, bv, bg);
            double dA = C.wu[qx] * C.wu[qz] * hx * hz;
            for (int c = 0; c < 2; ++c)
              for (int a = 0; a < 2; ++a) {
                double N = (a ? xi[0] : 1 - xi[0]) * (c ? xi[2] : 1 - xi[2]);
                int64_t node = ((int64_t)w * nz + (ez + c) % nz) * nx + (ex + a) % nx;
                for (int i = 0; i < 3; ++i) num[node * 3 + i] += N * dA * P->nu * vp.g[i][1] * ny_out;
                den[node] += N * dA;
              }
          }
      }
  }
  for (int64_t b = 0; b < (int64_t)2 * nz * nx; ++b)
    out[b] = sqrt(num[b * 3] * num[b * 3] + num[b * 3 + 1] * num[b * 3 + 1] + num[b * 3 + 2] * num[b * 3 + 2]) /
             den[b];
  free(num);
  free(den);
  free(bv);
  ctx_free(&C);
  return 0;
}

/* Physical point and Jacobian determinant (for geometry tests). */
int orc_cell_map(const orc_params *P, int64_t e, const double *xi, double *X, double *detJ) {
  ctx C;
  if (ctx_init(&C, P, NULL)) return -1;
  double J[3][3], Ji[3][3];
  cell_map(&C, e, xi, X, J);
  *detJ = inv3(J, Ji);
  ctx_free(&C);
  return 0;
}

/* Jacobians J[d][a] = dX_d / dxi_a of cell e at npts reference points (xi:
 * [npts][3]; J: [npts][9]). */
int orc_cell_jacobians(const orc_params *P, int64_t e, int64_t npts, const double *xi, double *J9) {
  ctx C;
  if (ctx_init(&C, P, NULL)) return -1;
  if (e < 0 || e >= C.ncell) { ctx_free(&C); return -2; }
  for (int64_t q = 0; q < npts; ++q) {
    double X[3], J[3][3];
    cell_map(&C, e, xi + 3 * q, X, J);
    for (int d = 0; d < 3; ++d)
      for (int a = 0; a < 3; ++a) J9[9 * q + 3 * d + a] = J[d][a];
  }
  ctx_free(&C);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Multiscale viscous operator (Sec. 2.2 and Sec. 4.2)                        */
/* ------------------------------------------------------------------------ */

/* Eddy viscosity of the RANS scale at reference point xi of enriched cell e
 * (eq. mix): nu_t = l_mix^2 |eps(u~)|, |eps| = sqrt(2 eps : eps), with the
 * mixing length l_mix = kappa y_DES (1 - exp(-y+/A+)) (eq. lmix), the smooth
 * DES limit y_DES = (y^-beta + (C_DES h)^-beta)^(-1/beta) (eq. ydes; written
 * as y C h / (y^beta + (C h)^beta)^(1/beta), which is 0 at the wall), and
 * h = dy_e / (k+1) the wall-normal cell width over k+1.  gt = grad u~ [c][d]
 * (u~ = psi sum_B N^l_B ut_B, so grad u~ = sum_B ut_B (x) grad(psi N^l_B)).
 * y = y_h (the wall distance of Sec. 3.2), y+ = y_h sqrt(tau_w)/nu.
 * out: nu_t, y, y+, |eps(u~)|.  Flat walls only. */
static void eddy_point(const ctx *C, int64_t e, const double xi[3], const double Ji[3][3], const double gt[3][3],
                       double c_des, double beta, double out[4]) {
  int ex, ey, ez;
  cell_index(C, e, &ex, &ey, &ez);
  double yh, gyh[3], tw, gtw[3];
  wall_fields(C, e, xi, Ji, &yh, gyh, &tw, gtw);
  double yp = yh * sqrt(tw) / C->P.nu;
  double h = (C->eta[ey + 1] - C->eta[ey]) / (C->P.k_u + 1);
  double ch = c_des * h;
  double ydes = yh * ch / pow(pow(yh, beta) + pow(ch, beta), 1.0 / beta);
  double lmix = C->P.kappa * ydes * (1.0 - exp(-yp / C->P.A_plus));
  double eps2 = 0;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double eij = 0.5 * (gt[i][j] + gt[j][i]);
      eps2 += eij * eij;
    }
  double em = sqrt(2.0 * eps2);
  out[0] = lmix * lmix * em;
  out[1] = yh;
  out[2] = yp;
  out[3] = em;
}

typedef struct {
  double ub[3], gb[3][3];  /* polynomial part u_bar and its gradient [c][d]     */
  double ut[3], gt[3][3];  /* enrichment part u~ and its gradient                 */
  double ev[8], eg[8][3];  /* enrichment functions psi N^l_B and their gradients  */
  double nut;              /* eddy viscosity (zero outside enriched cells)        */
  int enriched;
} ms_pt;

/* sum_B w_B f_B (x) grad: value and gradient of an enrichment field with
 * coefficients w[c][B] at a point with enrichment functions ev, eg. */
static void enr_field(int nle, const double *w, const double *ev, const double (*eg)[3], double v[3],
                      double g[3][3]) {
  for (int c = 0; c < 3; ++c) {
    v[c] = 0;
    for (int d = 0; d < 3; ++d) g[c][d] = 0;
    for (int B = 0; B < nle; ++B) {
      v[c] += ev[B] * w[c * nle + B];
      for (int d = 0; d < 3; ++d) g[c][d] += eg[B][d] * w[c * nle + B];
    }
  }
}

/* Both scales of the velocity at xi of cell e, and nu_t from the enrichment
 * coefficients of unut. */
static void eval_ms(const ctx *C, const double *u, const double *unut, int64_t e, const double xi[3],
                    const double Ji[3][3], double c_des, double beta, ms_pt *o, double *bv, double (*bg)[3]) {
  int n = C->npu, np3 = n * n * n;
  basis3(n, C->glu, xi, Ji, bv, bg);
  for (int c = 0; c < 3; ++c) {
    const double *uc = u + ((int64_t)e * 3 + c) * np3;
    double s = 0, g0 = 0, g1 = 0, g2 = 0;
    for (int B = 0; B < np3; ++B) {
      s += bv[B] * uc[B];
      g0 += bg[B][0] * uc[B];
      g1 += bg[B][1] * uc[B];
      g2 += bg[B][2] * uc[B];
    }
    o->ub[c] = s;
    o->gb[c][0] = g0; o->gb[c][1] = g1; o->gb[c][2] = g2;
    o->ut[c] = 0;
    for (int d = 0; d < 3; ++d) o->gt[c][d] = 0;
  }
  for (int B = 0; B < 8; ++B) {
    o->ev[B] = 0;
    for (int d = 0; d < 3; ++d) o->eg[B][d] = 0;
  }
  o->nut = 0;
  o->enriched = (C->enr[e] >= 0);
  if (!o->enriched) return;
  psi_pt ps;
  eval_psi(C, e, xi, Ji, &ps);
  enr_basis(C, xi, Ji, &ps, o->ev, o->eg);
  const int nle = C->nle;
  const double *ut = u + C->ncell * 3 * np3 + C->enr[e] * 3 * nle;
  const double *un = unut + C->ncell * 3 * np3 + C->enr[e] * 3 * nle;
  enr_field(nle, ut, o->ev, (const double(*)[3])o->eg, o->ut, o->gt);
  double vn[3], gn[3][3], out[4];
  enr_field(nle, un, o->ev, (const double(*)[3])o->eg, vn, gn);
  eddy_point(C, e, xi, Ji, (const double(*)[3])gn, c_des, beta, out);
  o->nut = out[0];
}

/* A(v, u) = -F^nu_e(v_bar, v~, u_bar, u~) of eq. viscous_multiscale for every
 * test function v of cell e (v_bar = N_B e_c; v~ = psi N^l_B e_c in an
 * enriched cell), with F^a(w) = 2 a eps(w) and, as the paper's rows and
 * columns read:
 *   volume:  (eps(v_bar), F^nu(u_bar))_e + (eps(v_bar), F^nuhat(u~))_e
 *            + (eps(v~), F^{nu+nu_t}(u~))_e,
 *            nuhat = min(nu + nu_t, 2 sqrt(nu (nu + nu_t))) (eq. minvt; clip = 0
 *            keeps nu + nu_t, for the coercivity pins only);
 *   faces, by class (own cell "-", outward n, [w] = w- - w+):
 *   regular (no enriched side): (1/2 F^nu(v_bar), [u_bar] (x) n)
 *            - (v_bar, {{F^nu(u_bar)}} n) + (v_bar, tau nu [u_bar]);
 *   interface (exactly one side enriched, u~ = 0 on the other):
 *            (1/2 F^nu(v_bar), [u] (x) n) - (v, {{F^nu(u_bar)}} n) + (v, tau nu [u])
 *            for v = v_bar, and the last two terms for v = v~;
 *   inner enriched (both sides enriched; a wall of an enriched cell, whose
 *   mirror side is enriched too):
 *            (1/2 F^nu(v_bar), [u_bar] (x) n) - (v_bar, {{F^nu(u_bar)}} n)
 *            - (v, {{F^{nu+nu_t}(u~)}}_w n) + (v, tau nu [u]) for v = v_bar, v~,
 *            and (w- F^{nu+nu_t}(v~), [u] (x) n) for v = v~,
 * with u = u_bar + u~, {{.}} the mean with weights 1/2 and {{.}}_w the
 * harmonic weights w- = (nu + nu_t+)/(2 nu + nu_t- + nu_t+), w+ = (nu +
 * nu_t-)/(2 nu + nu_t- + nu_t+) (eq. harmweights).  Walls: mirror data
 * u+ = -u-, grad u+ = grad u-, nu_t+ = nu_t-, tau x wall_ip_mult.  The
 * penalty carries nu alone and tau as in the velocity residual.  nu_t comes
 * from the enrichment coefficients of unut.  M du/dt = -A u is the viscous
 * substep of the paper's scheme. */
static void visc_ms_cell(const ctx *C, const double *u, const double *unut, int64_t e, double *r, double c_des,
                         double beta, int clip, double *bv, double (*bg)[3], double *bv2, double (*bg2)[3]) {
  int n = C->npu, np3 = n * n * n;
  double nu = C->P.nu;
  double *re = r + (int64_t)e * 3 * np3;
  const int nle = C->nle;
  double rt[3 * 8] = {0};  /* enrichment rows [c][B] */
  for (int i = 0; i < 3 * np3; ++i) re[i] = 0.0;
  int e_enr = C->enr[e] >= 0;

  /* volume */
  {
    const double *q[3], *w[3];
    int nq[3];
    for (int a = 0; a < 3; ++a) { q[a] = vel_q(C, e, a, &w[a]); nq[a] = vel_nq(C, e, a); }
    for (int c3 = 0; c3 < nq[2]; ++c3)
      for (int b = 0; b < nq[1]; ++b)
        for (int a = 0; a < nq[0]; ++a) {
          double xi[3] = {q[0][a], q[1][b], q[2][c3]}, X[3], J[3][3], Ji[3][3];
          cell_map(C, e, xi, X, J);
          double wq = fabs(inv3(J, Ji)) * w[0][a] * w[1][b] * w[2][c3];
          ms_pt p;
          eval_ms(C, u, unut, e, xi, Ji, c_des, beta, &p, bv, bg);
          double nt = nu + p.nut;
          double nhat = clip ? fmin(nt, 2.0 * sqrt(nu * nt)) : nt;
          for (int c = 0; c < 3; ++c) {
            double G[3];
            for (int d = 0; d < 3; ++d)
              G[d] = nu * (p.gb[c][d] + p.gb[d][c]) + nhat * (p.gt[c][d] + p.gt[d][c]);
            double *rc = re + c * np3;
            for (int B = 0; B < np3; ++B) rc[B] += wq * (bg[B][0] * G[0] + bg[B][1] * G[1] + bg[B][2] * G[2]);
            if (p.enriched)
              for (int B = 0; B < nle; ++B) {
                /* eps(phi e_c) : F = sum_d d_d phi F[c][d] for symmetric F, phi = psi N^l_B */
                double s = 0;
                for (int d = 0; d < 3; ++d) s += p.eg[B][d] * nt * (p.gt[c][d] + p.gt[d][c]);
                rt[c * nle + B] += wq * s;
              }
          }
        }
  }

  /* faces */
  double vol_e = cell_volume(C, e, 0);
  for (int f = 0; f < 6; ++f) {
    int d = f / 2, s = f % 2;
    int t1 = (d == 0) ? 1 : 0, t2 = (d == 2) ? 1 : 2;
    int64_t nb = face_neighbor(C, e, d, s);
    int wall = (nb < 0);
    int nb_enr = !wall && C->enr[nb] >= 0;
    int inner = e_enr && (wall || nb_enr);  /* otherwise an enriched cell's face is an interface */
    const double *q1, *w1, *q2, *w2;
    int n1, n2;
    face_rule(C, e, nb, t1, t2, &q1, &w1, &n1, &q2, &w2, &n2);
    double area = 0;
    for (int b = 0; b < n2; ++b)
      for (int a = 0; a < n1; ++a) {
        double xi[3], X[3], Ji[3][3], nv[3], dA;
        xi[d] = s; xi[t1] = q1[a]; xi[t2] = q2[b];
        face_point(C, e, d, s, xi, X, Ji, nv, &dA);
        area += dA * w1[a] * w2[b];
      }
    double pf = C->P.ip_factor_u * (double)(n) * (double)(n);
    double tauF = wall ? C->P.wall_ip_mult * pf * area / vol_e
                       : pf * fmax(area / vol_e, area / cell_volume(C, nb, 0));
    for (int b = 0; b < n2; ++b)
      for (int a = 0; a < n1; ++a) {
        double xi[3], xn[3], X[3], Ji[3][3], Xn[3], Jn[3][3], Jin[3][3], nv[3], dA;
        xi[d] = s; xi[t1] = q1[a]; xi[t2] = q2[b];
        face_point(C, e, d, s, xi, X, Ji, nv, &dA);
        double wf = dA * w1[a] * w2[b];
        ms_pt pm, pp;
        eval_ms(C, u, unut, e, xi, Ji, c_des, beta, &pm, bv, bg);
        if (wall) {
          pp = pm;
          for (int c = 0; c < 3; ++c) { pp.ub[c] = -pm.ub[c]; pp.ut[c] = -pm.ut[c]; }
        } else {
          xn[d] = 1 - s; xn[t1] = xi[t1]; xn[t2] = xi[t2];
          cell_map(C, nb, xn, Xn, Jn);
          inv3(Jn, Jin);
          eval_ms(C, u, unut, nb, xn, Jin, c_des, beta, &pp, bv2, bg2);
        }
        double jb[3], ju[3], Eb[3], Et[3];
        double wm = 0.5, wp = 0.5;
        if (inner) {
          double den = 2.0 * nu + pm.nut + pp.nut;
          wm = (nu + pp.nut) / den;
          wp = (nu + pm.nut) / den;
        }
        for (int c = 0; c < 3; ++c) {
          jb[c] = pm.ub[c] - pp.ub[c];
          ju[c] = (pm.ub[c] + pm.ut[c]) - (pp.ub[c] + pp.ut[c]);
          double sb = 0, st = 0;
          for (int k = 0; k < 3; ++k) {
            sb += 0.5 * nu * ((pm.gb[c][k] + pm.gb[k][c]) + (pp.gb[c][k] + pp.gb[k][c])) * nv[k];
            st += (wm * (nu + pm.nut) * (pm.gt[c][k] + pm.gt[k][c]) +
                   wp * (nu + pp.nut) * (pp.gt[c][k] + pp.gt[k][c])) * nv[k];
          }
          Eb[c] = sb;
          Et[c] = inner ? st : 0.0;
        }
        /* test functions N_B e_c */
        const double *J = inner ? jb : ju;
        for (int c = 0; c < 3; ++c) {
          double fv = -Eb[c] - Et[c] + tauF * nu * ju[c];
          double Fg[3];
          for (int k = 0; k < 3; ++k) Fg[k] = nu * 0.5 * (J[c] * nv[k] + J[k] * nv[c]);
          double *rc = re + c * np3;
          for (int B = 0; B < np3; ++B)
            rc[B] += wf * (bv[B] * fv + bg[B][0] * Fg[0] + bg[B][1] * Fg[1] + bg[B][2] * Fg[2]);
        }
        /* test functions phi e_c, phi = psi N^l_B */
        if (e_enr)
          for (int B = 0; B < nle; ++B) {
            const double *gp = pm.eg[B];
            double gn = gp[0] * nv[0] + gp[1] * nv[1] + gp[2] * nv[2];
            double jg = ju[0] * gp[0] + ju[1] * gp[1] + ju[2] * gp[2];
            for (int c = 0; c < 3; ++c) {
              double val;
              if (inner)
                val = pm.ev[B] * (-Et[c] + tauF * nu * ju[c]) + wm * (nu + pm.nut) * (ju[c] * gn + jg * nv[c]);
              else /* interface */
                val = pm.ev[B] * (-Eb[c] + tauF * nu * ju[c]);
              rt[c * nle + B] += wf * val;
            }
          }
      }
  }
  if (e_enr) {
    double *ro = r + C->ncell * 3 * np3 + C->enr[e] * 3 * nle;
    for (int i = 0; i < 3 * nle; ++i) ro[i] = rt[i];
  }
}

int orc_viscous_multiscale(const orc_params *P, const double *u, const double *u_nut, const double *tau_w,
                           const double *tau_nodes, double c_des, double beta, int clip, const int64_t *cells,
                           int64_t ncells, double *r) {
  ctx C;
  if (ctx_init(&C, P, tau_w)) return -1;
  C.tau_nodes = tau_nodes;
  if (C.nenr > 0 && !tau_w && !tau_nodes) { ctx_free(&C); return -2; }
  if (P->wall_amp != 0.0) { ctx_free(&C); return -4; }
  ctx_activity(&C, -1);
  int n = C.npu, np3 = n * n * n;
  int err = 0;
#pragma omp parallel
  {
    double *bv = (double *)malloc(sizeof(double) * np3 * 2);
    double(*bg)[3] = (double(*)[3])malloc(sizeof(double) * 3 * np3 * 2);
#pragma omp for schedule(dynamic, 4)
    for (int64_t i = 0; i < ncells; ++i) {
      int64_t e = cells[i];
      if (e < 0 || e >= C.ncell) { err = -3; continue; }
      visc_ms_cell(&C, u, u_nut, e, r, c_des, beta, clip, bv, bg, bv + np3, bg + np3);
    }
    free(bv);
    free(bg);
  }
  ctx_free(&C);
  return err;
}

/* nu_t, y, y+ and |eps(u~)| at reference point xi of enriched cell e, with the
 * enrichment coefficients of u_nut (see eddy_point).  Returns -2 for a cell
 * without enrichment. */
int orc_eddy_viscosity_point(const orc_params *P, const double *u_nut, const double *tau_w, const double *tau_nodes,
                             double c_des, double beta, int64_t e, const double *xi, double *out4) {
  ctx C;
  if (ctx_init(&C, P, tau_w)) return -1;
  C.tau_nodes = tau_nodes;
  if (e < 0 || e >= C.ncell || C.enr[e] < 0 || P->wall_amp != 0.0) { ctx_free(&C); return -2; }
  ctx_activity(&C, -1);
  double X[3], J[3][3], Ji[3][3];
  cell_map(&C, e, xi, X, J);
  inv3(J, Ji);
  psi_pt ps;
  eval_psi(&C, e, xi, Ji, &ps);
  int np3 = C.npu * C.npu * C.npu;
  double ev[8], eg[8][3], vn[3], gn[3][3];
  enr_basis(&C, xi, Ji, &ps, ev, eg);
  enr_field(C.nle, u_nut + C.ncell * 3 * np3 + C.enr[e] * 3 * C.nle, ev, (const double(*)[3])eg, vn, gn);
  eddy_point(&C, e, xi, Ji, (const double(*)[3])gn, c_des, beta, out4);
  ctx_free(&C);
  return 0;
}

/* Quadrature points of face f = 2 d + s of cell e with the face rule of the
 * velocity residual (the larger tangential counts of the two adjacent cells).
 * Per point, 7 doubles: X[3], n w dA [3] (outward unit normal times weight
 * times area element) and w dA.  out holds 7 ORC_MAXN^2 doubles; returns the
 * number of points, negative on bad arguments. */
int orc_face_points(const orc_params *P, int64_t e, int f, double *out) {
  ctx C;
  if (ctx_init(&C, P, NULL)) return -1;
  if (e < 0 || e >= C.ncell || f < 0 || f > 5) { ctx_free(&C); return -2; }
  int d = f / 2, s = f % 2;
  int t1 = (d == 0) ? 1 : 0, t2 = (d == 2) ? 1 : 2;
  int64_t nb = face_neighbor(&C, e, d, s);
  const double *q1, *w1, *q2, *w2;
  int n1, n2;
  face_rule(&C, e, nb, t1, t2, &q1, &w1, &n1, &q2, &w2, &n2);
  int np = 0;
  for (int b = 0; b < n2; ++b)
    for (int a = 0; a < n1; ++a) {
      double xi[3], X[3], Ji[3][3], nv[3], dA;
      xi[d] = s; xi[t1] = q1[a]; xi[t2] = q2[b];
      face_point(&C, e, d, s, xi, X, Ji, nv, &dA);
      double wf = dA * w1[a] * w2[b];
      double *o = out + 7 * np++;
      for (int k = 0; k < 3; ++k) { o[k] = X[k]; o[3 + k] = nv[k] * wf; }
      o[6] = wf;
    }
  ctx_free(&C);
  return np;
}

/* Number of OpenMP threads the oracle uses (for reporting). */
int orc_num_threads(void) {
  int n = 1;
#pragma omp parallel
  {
#pragma omp single
    n = omp_get_num_threads();
  }
  return n;
}
