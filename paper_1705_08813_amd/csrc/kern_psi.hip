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
// The tables are computed once per wall-shear update and stored, as the
// paper does for its enrichment.
#include "kern_common.h"

namespace dgwm {

namespace {

// Safeguarded Newton for Spalding's law.  f(U) is increasing and convex on
// U >= 0 with f(0) = -y+ <= 0 <= f(y+), so [0, y+] brackets the root; steps
// leaving the bracket fall back to bisection.
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
    double xn = x - f / df;
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

// pts: the NQ Gauss points of the wall-parallel rule followed by the NQY
// points of the wall-normal rule (on [0,1]).
// Curved lower wall: y_h is the bilinear (x, eta) interpolation of the vertex
// distances to the closest wall vertex (wdist: rows iy = 1 and iy = ny-1; the
// wall rows are 0), grad y_h = J^{-T} grad_xi y_h with J^{-1} from the
// geometry table at the same point.
template <int NQ, int NQY>
__global__ void psi_kernel(int nx, int ny, int nz, int lower_slot, int nslots, const double* __restrict__ eta,
                           const double* __restrict__ pts, const double* __restrict__ tau, double nu, double kappa,
                           double B, int64_t nenr, int psi_pts, double* __restrict__ psi,
                           const double* __restrict__ geo, int geo_stride, const double* __restrict__ wdist,
                           int psi_kind, double A_plus, const VdTable vd, const double* __restrict__ tau_nodes,
                           double hx, double hz) {
  constexpr int NPTS = NQ * NQY * NQ;
  const int64_t gid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (gid >= nenr * psi_pts) return;
  const int64_t enr = gid / psi_pts;
  const int pt = (int)(gid - enr * psi_pts);
  const int ex = (int)(enr % nx);
  const int64_t t0 = enr / nx;
  const int slot = (int)(t0 % nslots);
  const int ez = (int)(t0 / nslots);
  const bool lower = (slot == lower_slot);
  const int ey = lower ? 0 : ny - 1;
  const double* gy = pts + NQ;
  // reference coordinates of the point and its tau column
  double xiy, xix, xiz;
  int qx, qz;
  if (pt < NPTS) {
    qx = pt % NQ;
    xix = pts[qx];
    xiy = gy[(pt / NQ) % NQY];
    qz = pt / (NQ * NQY);
    xiz = pts[qz];
  } else {
    int f = 0, o = NPTS;
    while (pt >= o + psi_face_points(NQ, NQY, f / 2)) {
      o += psi_face_points(NQ, NQY, f / 2);
      ++f;
    }
    const int d = f / 2, s = f % 2, k = pt - o;
    const int Q1 = d == 0 ? NQY : NQ;  // first tangential direction: y for x-faces, x otherwise
    const int q1 = k % Q1, q2 = k / Q1;
    if (d == 0) {
      qx = s ? NQ - 1 : 0;
      xix = (double)s;
      xiy = gy[q1];
      qz = q2;
      xiz = pts[q2];
    } else if (d == 1) {
      qx = q1;
      xix = pts[q1];
      xiy = (double)s;
      qz = q2;
      xiz = pts[q2];
    } else {
      qx = q1;
      xix = pts[q1];
      xiy = gy[q2];
      qz = s ? NQ - 1 : 0;
      xiz = (double)s;
    }
  }
  double yh, gyh[3];
  if (!geo) {
    const double y = eta[ey] + (eta[ey + 1] - eta[ey]) * xiy;
    yh = lower ? y + 1.0 : 1.0 - y;
    gyh[0] = 0.0;
    gyh[1] = lower ? 1.0 : -1.0;
    gyh[2] = 0.0;
  } else {
    const double d00 = lower ? 0.0 : wdist[nx + 1 + ex], d10 = lower ? 0.0 : wdist[nx + 1 + ex + 1];
    const double d01 = lower ? wdist[ex] : 0.0, d11 = lower ? wdist[ex + 1] : 0.0;
    const double bot = (1.0 - xix) * d00 + xix * d10, top = (1.0 - xix) * d01 + xix * d11;
    yh = (1.0 - xiy) * bot + xiy * top;
    const double gx = (1.0 - xiy) * (d10 - d00) + xiy * (d11 - d01), gyy = top - bot;
    const int64_t e = ex + (int64_t)nx * (ey + (int64_t)ny * ez);
    const double* Ji = geo + (e * geo_stride + pt) * 10;
    for (int dd = 0; dd < 3; ++dd) gyh[dd] = gx * Ji[0 * 3 + dd] + gyy * Ji[1 * 3 + dd];
  }
  const int w = lower ? 0 : 1;
  double tw, gtx = 0.0, gtz = 0.0;
  if (tau_nodes) {
    // wall vertices (ex, ez) .. (ex+1, ez+1) on the periodic vertex grid
    const double* tn = tau_nodes + (int64_t)w * nz * nx;
    const int jx = ex + 1 == nx ? 0 : ex + 1, jz = ez + 1 == nz ? 0 : ez + 1;
    const double t00 = tn[(int64_t)ez * nx + ex], t10 = tn[(int64_t)ez * nx + jx];
    const double t01 = tn[(int64_t)jz * nx + ex], t11 = tn[(int64_t)jz * nx + jx];
    tw = (1.0 - xiz) * ((1.0 - xix) * t00 + xix * t10) + xiz * ((1.0 - xix) * t01 + xix * t11);
    gtx = ((1.0 - xiz) * (t10 - t00) + xiz * (t11 - t01)) / hx;
    gtz = ((1.0 - xix) * (t01 - t00) + xix * (t11 - t10)) / hz;
  } else {
    tw = tau[(((int64_t)w * nz + ez) * nx + ex) * NQ * NQ + (int64_t)qz * NQ + qx];
  }
  double* o = psi + gid * 4;
  if (!(tw > 0.0) || !isfinite(tw)) {
    o[0] = o[1] = o[2] = o[3] = __builtin_nan("");
    return;
  }
  const double st = sqrt(tw) / nu;
  double U, dU;
  if (psi_kind == DG_PSI_VANDRIEST)
    vandriest_eval(fmax(yh, 0.0) * st, kappa, A_plus, vd, U, dU);
  else
    spalding_root(fmax(yh, 0.0) * st, kappa, B, U, dU);
  // y+ depends on tau_w through sqrt(tau_w): d y+/d tau_w = y_h / (2 nu sqrt(tau_w))
  const double dt = yh / (2.0 * nu * sqrt(tw));
  o[0] = U;
  o[1] = dU * st * gyh[0] + dU * dt * gtx;
  o[2] = dU * st * gyh[1];
  o[3] = dU * st * gyh[2] + dU * dt * gtz;
}

}  // namespace

#define DG_PSI_COMBOS(X) X(4, 8) X(4, 4) X(5, 8) X(5, 5) X(7, 8) X(8, 8)

int launch_psi(const dg_mesh* m, hipStream_t s) {
  if (m->nenr == 0) return DG_OK;
  // the Gauss points of both rules, contiguous, right after the tables
  const double* pts = m->tab_u + tab_layout(m->np_u, m->P.nq_u, m->P.nq_wn).size;
  const int64_t n = m->nenr * m->psi_pts;
  const unsigned nb = (unsigned)((n + 127) / 128);
  const int lower_slot = m->lower_slot;
#define X(a, b)                                                                                              \
  if (m->P.nq_u == a && m->P.nq_wn == b) {                                                                   \
    hipLaunchKernelGGL((psi_kernel<a, b>), dim3(nb), dim3(128), 0, s, m->P.nx, m->P.ny, m->P.nz, lower_slot, \
                       m->n_enr_layers, m->eta, pts, m->tau, m->P.nu, m->P.kappa, m->P.B, m->nenr,          \
                       m->psi_pts, m->psi, m->geo, m->geo_stride, m->wdist, m->P.psi_kind, m->P.A_plus,      \
                       m->vd, m->tau_nodal ? m->tau_nodes : nullptr, m->hx, m->hz);                          \
    return check_hip(hipGetLastError(), "psi kernel launch");                                                \
  }
  DG_PSI_COMBOS(X)
#undef X
  return set_error(DG_ERR_UNSUPPORTED, "psi table: quadrature combination not compiled");
}

}  // namespace dgwm
