// Enrichment function psi and its gradient at every quadrature point of the
// enriched cells (arXiv 1705.08813, Sec. 3.2), FP64.
//
//   y+ = y_h sqrt(tau_w) / nu    (rho = 1)
//   psi = U(y+) with U the root of Spalding's law
//         y+ = U + exp(-kappa B) (exp(kappa U) - 1 - kappa U - (kappa U)^2/2 - (kappa U)^3/6)
//   or van Driest's law (eq. psi), U = int_0^{y+} 2 ds / (1 + sqrt(1 + (2 kappa s (1 - exp(-s/A+)))^2))
//   grad psi = U'(y+) sqrt(tau_w)/nu grad y_h
//
// y_h is the wall distance (flat walls: exact, since the linear interpolation
// of the vertex distances is exact there).  tau_w comes from one of two
// fields:
//  - per point: the value of the wall-face Gauss column nearest to the point
//    (piecewise constant over the cell's wall footprint, zero gradient);
//  - nodal (flat walls): tau_w,h = sum_B N_B tau_w,B with the bilinear hats of
//    the wall vertices, constant along the wall normal, and the chain rule
//    grad y+ = sqrt(tau_w)/nu grad y_h + y_h/(2 nu sqrt(tau_w)) grad tau_w.
// Switch-off (Sec. 3.2): the enrichment of a cell is off while every point
// of its volume rule has y+ below yplus_off; such a cell gets psi = 0 and
// grad psi = 0, and its flag in the activity array is 0.
// The tables are computed once per wall-shear update and stored, as the
// paper does for its enrichment.
#include "kern_common.h"

namespace dgwm {

namespace {

// Safeguarded Halley iteration for Spalding's law.  f(U) is increasing and
// convex on U >= 0 with f(0) = -y+ <= 0 <= f(y+), so [0, y+] brackets the
// root; the cubic step x - f f' / (f'^2 - f f''/2) (f'' = c kappa^2 (e^k - 1
// - k) costs nothing beyond the exponential already formed) falls back to
// Newton where its denominator is not positive and to bisection where a step
// leaves the bracket.
__device__ void spalding_root(double yp, double kappa, double B, double& U, double& dU) {
  const double c = exp(-kappa * B);
  double lo = 0.0, hi = yp;
  double x = yp < 10.0 ? yp : fmin(yp, log(yp) / kappa + B);
  for (int it = 0; it < 100; ++it) {
    const double k = kappa * x;
    const double em1 = expm1(k);
    const double f = x + c * (em1 - k - 0.5 * k * k - k * k * k / 6.0) - yp;
    if (f == 0.0) break;
    if (f > 0.0) hi = x; else lo = x;
    const double df = 1.0 + c * kappa * (em1 - k - 0.5 * k * k);
    const double d2f = c * kappa * kappa * (em1 - k);
    const double den = df * df - 0.5 * f * d2f;
    double xn = den > 0.0 ? x - f * df / den : x - f / df;
    if (!(xn >= lo && xn <= hi)) xn = 0.5 * (lo + hi);
    const double step = fabs(xn - x);
    x = xn;
    if (step <= 4e-16 * fmax(1.0, x)) break;
  }
  const double k = kappa * x;
  U = x;
  dU = 1.0 / (1.0 + c * kappa * (expm1(k) - k - 0.5 * k * k));
}

// van Driest's law (Sec. 3.2, eq. psi) as in the paper's Appendix A: U at
// the support point y+_i below y+ comes from the set-up table, the slice
// [y+_i, y+] is integrated with the 9-point Gauss rule; dU/dy+ is the
// integrand f(s) = 2 / (1 + sqrt(1 + (2 kappa s (1 - exp(-s/A+)))^2)).
__device__ __forceinline__ double vandriest_f(double s, double kappa, double Ap) {
  const double m = 2.0 * kappa * s * (-expm1(-s / Ap));
  return 2.0 / (1.0 + sqrt(1.0 + m * m));
}

__device__ void vandriest_eval(double yp, double kappa, double Ap, const VdTable& tb, double& U, double& dU) {
  constexpr auto& G = ct::tab<2, 9>;  // 9-point Gauss rule on [0,1] (the basis part is unused)
  int i = 0;
#pragma unroll
  for (int j = 1; j < VdTable::N; ++j)
    if (tb.y[j] <= yp) i = j;
  const double a = tb.y[i], h = yp - a;
  double sum = 0.0;
#pragma unroll
  for (int q = 0; q < 9; ++q) sum += G.w[q] * vandriest_f(a + h * G.g[q], kappa, Ap);
  U = tb.psi[i] + h * sum;
  dU = vandriest_f(yp, kappa, Ap);
}

// Everything the point evaluations read.  pts: the NQ Gauss points of the
// wall-parallel rule followed by the NQY points of the wall-normal rule (on
// [0,1]).
struct PsiArgs {
  int nx, ny, nz, lower_slot, nslots, psi_pts, geo_stride, psi_kind;
  int64_t nenr;
  const double* eta;
  const double* pts;
  const double* tau;        // per wall-face Gauss point
  const double* tau_nodes;  // or nodal [wall][nz][nx] (nullptr: per point)
  const double* geo;        // curved: [cell][point][J^{-1}, weight]; nullptr: flat
  const double* wdist;      // curved: [2][nx+1] wall-adjacent vertex distances
  double nu, kappa, B, A_plus, hx, hz, yplus_off;
  double* psi;
  int32_t* act;
  VdTable vd;
};

struct CellRef {
  int ex, ey, ez, w;  // w: 0 lower wall, 1 upper wall
  bool lower;
};

// (the enriched count stays below 2^31 like the cell count, so 32-bit
// division suffices)
__device__ __forceinline__ CellRef enriched_cell(const PsiArgs& A, int64_t enr64) {
  CellRef c;
  const int enr = (int)enr64;
  c.ex = enr % A.nx;
  const int t0 = enr / A.nx;
  const int slot = (int)(t0 % A.nslots);
  c.ez = (int)(t0 / A.nslots);
  c.lower = (slot == A.lower_slot);
  c.ey = c.lower ? 0 : A.ny - 1;
  c.w = c.lower ? 0 : 1;
  return c;
}

// Reference coordinates of point pt of the psi tables (volume rule, then the
// six faces) and the wall-face Gauss column (qx, qz) nearest to it.
struct PointRef {
  double xix, xiy, xiz;
  int qx, qz;
};

template <int NQ, int NQY>
__device__ __forceinline__ PointRef decode_point(int pt, const double* pts) {
  constexpr int NPTS = NQ * NQY * NQ;
  const double* gy = pts + NQ;
  PointRef r;
  if (pt < NPTS) {
    r.qx = pt % NQ;
    r.xix = pts[r.qx];
    r.xiy = gy[(pt / NQ) % NQY];
    r.qz = pt / (NQ * NQY);
    r.xiz = pts[r.qz];
    return r;
  }
  int f = 0, o = NPTS;
  while (pt >= o + psi_face_points(NQ, NQY, f / 2)) {
    o += psi_face_points(NQ, NQY, f / 2);
    ++f;
  }
  const int d = f / 2, s = f % 2, k = pt - o;
  const int Q1 = d == 0 ? NQY : NQ;  // first tangential direction: y for x-faces, x otherwise
  const int q1 = k % Q1, q2 = k / Q1;
  if (d == 0) {
    r.qx = s ? NQ - 1 : 0;
    r.xix = (double)s;
    r.xiy = gy[q1];
    r.qz = q2;
    r.xiz = pts[q2];
  } else if (d == 1) {
    r.qx = q1;
    r.xix = pts[q1];
    r.xiy = (double)s;
    r.qz = q2;
    r.xiz = pts[q2];
  } else {
    r.qx = q1;
    r.xix = pts[q1];
    r.xiy = gy[q2];
    r.qz = s ? NQ - 1 : 0;
    r.xiz = (double)s;
  }
  return r;
}

// Wall distance y_h at the point and, when gyh != nullptr, its physical
// gradient.  Curved lower wall: y_h is the bilinear (x, eta) interpolation
// of the vertex distances to the closest wall vertex (wdist: rows iy = 1 and
// iy = ny-1; the wall rows are 0), grad y_h = J^{-T} grad_xi y_h with J^{-1}
// from the geometry table at the same point (index pt).
__device__ __forceinline__ double wall_distance(const PsiArgs& A, const CellRef& c, const PointRef& p, int pt,
                                                double* gyh) {
  if (!A.geo) {
    const double y = A.eta[c.ey] + (A.eta[c.ey + 1] - A.eta[c.ey]) * p.xiy;
    if (gyh) {
      gyh[0] = 0.0;
      gyh[1] = c.lower ? 1.0 : -1.0;
      gyh[2] = 0.0;
    }
    return c.lower ? y + 1.0 : 1.0 - y;
  }
  const int nx = A.nx, ex = c.ex;
  const double d00 = c.lower ? 0.0 : A.wdist[nx + 1 + ex], d10 = c.lower ? 0.0 : A.wdist[nx + 1 + ex + 1];
  const double d01 = c.lower ? A.wdist[ex] : 0.0, d11 = c.lower ? A.wdist[ex + 1] : 0.0;
  const double bot = (1.0 - p.xix) * d00 + p.xix * d10, top = (1.0 - p.xix) * d01 + p.xix * d11;
  if (gyh) {
    const double gx = (1.0 - p.xiy) * (d10 - d00) + p.xiy * (d11 - d01), gyy = top - bot;
    const int64_t e = ex + (int64_t)nx * (c.ey + (int64_t)A.ny * c.ez);
    const double* Ji = A.geo + (e * A.geo_stride + pt) * 10;
    for (int dd = 0; dd < 3; ++dd) gyh[dd] = gx * Ji[0 * 3 + dd] + gyy * Ji[1 * 3 + dd];
  }
  return (1.0 - p.xiy) * bot + p.xiy * top;
}

// tau_w at the point: the nearest Gauss column of the per-point field (zero
// gradient), or the bilinear interpolation of the nodal field of the cell's
// four wall vertices (periodic vertex grid) with its gradient (gtx, gtz).
__device__ __forceinline__ double wall_tau(const PsiArgs& A, const CellRef& c, const PointRef& p, int NQ,
                                           double& gtx, double& gtz) {
  gtx = gtz = 0.0;
  if (!A.tau_nodes)
    return A.tau[(((int64_t)c.w * A.nz + c.ez) * A.nx + c.ex) * NQ * NQ + (int64_t)p.qz * NQ + p.qx];
  const double* tn = A.tau_nodes + (int64_t)c.w * A.nz * A.nx;
  const int jx = c.ex + 1 == A.nx ? 0 : c.ex + 1, jz = c.ez + 1 == A.nz ? 0 : c.ez + 1;
  const double t00 = tn[(int64_t)c.ez * A.nx + c.ex], t10 = tn[(int64_t)c.ez * A.nx + jx];
  const double t01 = tn[(int64_t)jz * A.nx + c.ex], t11 = tn[(int64_t)jz * A.nx + jx];
  gtx = ((1.0 - p.xiz) * (t10 - t00) + p.xiz * (t11 - t01)) / A.hx;
  gtz = ((1.0 - p.xix) * (t01 - t00) + p.xix * (t11 - t10)) / A.hz;
  return (1.0 - p.xiz) * ((1.0 - p.xix) * t00 + p.xix * t10) + p.xiz * ((1.0 - p.xix) * t01 + p.xix * t11);
}

// Switch-off rule (Sec. 3.2): the enrichment of a wall cell stays on while at
// least one point of its volume rule has y+ = y_h sqrt(tau_w)/nu >= yplus_off.
// One 64-lane workgroup per enriched cell, the points spread over the lanes.
template <int NQ, int NQY>
__global__ __launch_bounds__(64) void activity_kernel(const PsiArgs A) {
  constexpr int NPTS = NQ * NQY * NQ;
  const int64_t enr = blockIdx.x;
  const CellRef c = enriched_cell(A, enr);
  int on = 0;
  for (int pt = threadIdx.x; pt < NPTS; pt += 64) {
    const PointRef p = decode_point<NQ, NQY>(pt, A.pts);
    double gtx, gtz;
    const double yh = wall_distance(A, c, p, pt, nullptr);
    const double tw = wall_tau(A, c, p, NQ, gtx, gtz);
    if (yh * sqrt(tw) / A.nu >= A.yplus_off) on = 1;
  }
  on = __syncthreads_or(on);
  if (threadIdx.x == 0) A.act[enr] = on;
}

// psi, grad psi at every point of the tables; zeros in switched-off cells.
template <int NQ, int NQY>
__global__ void psi_kernel(const PsiArgs A) {
  const int64_t gid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (gid >= A.nenr * A.psi_pts) return;
  constexpr int PTS = psi_points(NQ, NQY);  // == A.psi_pts; a constant divisor
  const int64_t enr = gid / PTS;
  const int pt = (int)(gid - enr * PTS);
  double* o = A.psi + gid * 4;
  if (!A.act[enr]) {
    o[0] = o[1] = o[2] = o[3] = 0.0;
    return;
  }
  const CellRef c = enriched_cell(A, enr);
  const PointRef p = decode_point<NQ, NQY>(pt, A.pts);
  double gyh[3], gtx, gtz;
  const double yh = wall_distance(A, c, p, pt, gyh);
  const double tw = wall_tau(A, c, p, NQ, gtx, gtz);
  if (!(tw > 0.0) || !isfinite(tw)) {
    o[0] = o[1] = o[2] = o[3] = __builtin_nan("");
    return;
  }
  const double nu = A.nu;
  const double st = sqrt(tw) / nu;
  double U, dU;
  if (A.psi_kind == DG_PSI_VANDRIEST)
    vandriest_eval(fmax(yh, 0.0) * st, A.kappa, A.A_plus, A.vd, U, dU);
  else
    spalding_root(fmax(yh, 0.0) * st, A.kappa, A.B, U, dU);
  // y+ depends on tau_w through sqrt(tau_w): d y+/d tau_w = y_h / (2 nu sqrt(tau_w))
  const double dt = yh / (2.0 * nu * sqrt(tw));
  o[0] = U;
  o[1] = dU * st * gyh[0] + dU * dt * gtx;
  o[2] = dU * st * gyh[1];
  o[3] = dU * st * gyh[2] + dU * dt * gtz;
}

// Eddy viscosity of the RANS scale (Sec. 2.2) at every point of the psi
// tables: nu_t = l_mix^2 |eps(u~)| (eq. mix), l_mix = kappa y_DES (1 -
// exp(-y+/A+)) (eq. lmix), y_DES = y C h / (y^beta + (C h)^beta)^(1/beta), the
// smooth minimum of eq. ydes written so that it is 0 at the wall, h = dy_e /
// (k+1).  With l = 0, grad u~ = ut (x) grad psi (ut the cell's enrichment
// coefficients); with l = 1, grad u~ = sum_B ut_B (x) (N_B grad psi + psi
// grad N_B) over the trilinear vertex functions N_B of the cell (Sec. 3.1,
// eq. enrichment).  |eps| = sqrt(2 eps : eps).  Zero in switched-off cells.
struct EddyArgs {
  const double* ut;  // enrichment block of the velocity, [enr][c][B]
  double c_des, beta, inv_np;
  double* nut;
  int nle;           // enrichment functions per component: 1 (l = 0) or 8 (l = 1)
};

template <int NQ, int NQY>
__global__ void eddy_kernel(const PsiArgs A, const EddyArgs X) {
  const int64_t gid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (gid >= A.nenr * A.psi_pts) return;
  constexpr int PTS = psi_points(NQ, NQY);
  const int64_t enr = gid / PTS;
  const int pt = (int)(gid - enr * PTS);
  if (!A.act[enr]) {
    X.nut[gid] = 0.0;
    return;
  }
  const CellRef c = enriched_cell(A, enr);
  const PointRef p = decode_point<NQ, NQY>(pt, A.pts);
  double gtx, gtz;
  const double yh = fmax(wall_distance(A, c, p, pt, nullptr), 0.0);
  const double tw = wall_tau(A, c, p, NQ, gtx, gtz);
  const double yp = yh * sqrt(tw) / A.nu;
  const double ch = X.c_des * (A.eta[c.ey + 1] - A.eta[c.ey]) * X.inv_np;
  const double ydes = yh * ch / pow(pow(yh, X.beta) + pow(ch, X.beta), 1.0 / X.beta);
  const double lmix = A.kappa * ydes * (1.0 - exp(-yp / A.A_plus));
  const double* g = A.psi + gid * 4 + 1;
  double e2 = 0.0;
  if (X.nle == 1) {
    const double* ut = X.ut + enr * 3;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        const double eij = 0.5 * (ut[i] * g[j] + ut[j] * g[i]);
        e2 += eij * eij;
      }
  } else {
    const double* ut = X.ut + enr * 24;
    const double ps = A.psi[gid * 4];
    const double ih[3] = {1.0 / A.hx, 1.0 / (A.eta[c.ey + 1] - A.eta[c.ey]), 1.0 / A.hz};
    const double v[3][2] = {{1.0 - p.xix, p.xix}, {1.0 - p.xiy, p.xiy}, {1.0 - p.xiz, p.xiz}};
    double gt[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
#pragma unroll
    for (int B = 0; B < 8; ++B) {
      const int bx = B & 1, by = (B >> 1) & 1, bz = B >> 2;
      const double n = v[0][bx] * v[1][by] * v[2][bz];
      const double dn[3] = {(bx ? ih[0] : -ih[0]) * v[1][by] * v[2][bz], (by ? ih[1] : -ih[1]) * v[0][bx] * v[2][bz],
                            (bz ? ih[2] : -ih[2]) * v[0][bx] * v[1][by]};
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) gt[i][j] += ut[i * 8 + B] * (n * g[j] + ps * dn[j]);
    }
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        const double eij = 0.5 * (gt[i][j] + gt[j][i]);
        e2 += eij * eij;
      }
  }
  X.nut[gid] = lmix * lmix * sqrt(2.0 * e2);
}

}  // namespace

#define DG_PSI_COMBOS(X) X(4, 8) X(4, 4) X(5, 8) X(5, 5) X(7, 8) X(8, 8)

static PsiArgs psi_args(const dg_mesh* m) {
  PsiArgs A;
  A.nx = m->P.nx;
  A.ny = m->P.ny;
  A.nz = m->P.nz;
  A.lower_slot = m->lower_slot;
  A.nslots = m->n_enr_layers;
  A.psi_pts = m->psi_pts;
  A.geo_stride = m->geo_stride;
  A.psi_kind = m->P.psi_kind;
  A.nenr = m->nenr;
  A.eta = m->eta;
  // the Gauss points of both rules, contiguous, right after the tables
  A.pts = m->tab_u + tab_layout(m->np_u, m->P.nq_u, m->P.nq_wn).size;
  A.tau = m->tau;
  A.tau_nodes = m->tau_nodal ? m->tau_nodes : nullptr;
  A.geo = m->geo;
  A.wdist = m->wdist;
  A.nu = m->P.nu;
  A.kappa = m->P.kappa;
  A.B = m->P.B;
  A.A_plus = m->P.A_plus;
  A.hx = m->hx;
  A.hz = m->hz;
  A.yplus_off = m->P.yplus_off;
  A.psi = m->psi;
  A.act = m->act;
  A.vd = m->vd;
  return A;
}

int launch_psi(const dg_mesh* m, hipStream_t s) {
  if (m->nenr == 0) return DG_OK;
  const PsiArgs A = psi_args(m);
  const int64_t n = m->nenr * m->psi_pts;
  const unsigned nb = (unsigned)((n + 127) / 128);
#define X(a, b)                                                                            \
  if (m->P.nq_u == a && m->P.nq_wn == b) {                                                 \
    if (A.yplus_off > 0.0) {                                                               \
      hipLaunchKernelGGL((activity_kernel<a, b>), dim3((unsigned)m->nenr), dim3(64), 0, s, A); \
      int rc = check_hip(hipGetLastError(), "enrichment activity kernel launch");         \
      if (rc) return rc;                                                                   \
    }                                                                                      \
    hipLaunchKernelGGL((psi_kernel<a, b>), dim3(nb), dim3(128), 0, s, A);                  \
    return check_hip(hipGetLastError(), "psi kernel launch");                              \
  }
  DG_PSI_COMBOS(X)
#undef X
  return set_error(DG_ERR_UNSUPPORTED, "psi table: quadrature combination not compiled");
}

int launch_eddy_viscosity(const dg_mesh* m, const double* u, double c_des, double beta, double* nut, hipStream_t s) {
  if (m->nenr == 0) return DG_OK;
  const PsiArgs A = psi_args(m);
  EddyArgs X;
  X.ut = u + m->ncell * 3 * (int64_t)m->np_u * m->np_u * m->np_u;
  X.c_des = c_des;
  X.beta = beta;
  X.inv_np = 1.0 / m->np_u;
  X.nut = nut;
  X.nle = m->nle;
  const int64_t n = m->nenr * m->psi_pts;
  const unsigned nb = (unsigned)((n + 127) / 128);
#define X_(a, b)                                                                 \
  if (m->P.nq_u == a && m->P.nq_wn == b) {                                       \
    hipLaunchKernelGGL((eddy_kernel<a, b>), dim3(nb), dim3(128), 0, s, A, X);   \
    return check_hip(hipGetLastError(), "eddy viscosity kernel launch");        \
  }
  DG_PSI_COMBOS(X_)
#undef X_
  return set_error(DG_ERR_UNSUPPORTED, "eddy viscosity: quadrature combination not compiled");
}

}  // namespace dgwm
