// Curved-wall geometry: per-quadrature-point inverse Jacobians and weights,
// cell volumes, face areas and interior-penalty parameters.
//
// Geometry (the periodic-hill-like configuration of the workload, a stand-in
// for the paper's Sec. 5.2 geometry): lower wall y_w(x) = -1 + a cos(2 pi x/Lx),
// upper wall y = +1; every column between them is stretched linearly in the
// wall-normal vertex parameter eta.  Each cell is mapped isoparametrically
// with degree k_u through its Gauss-Lobatto points (x and z are affine, y(x, eta)
// is interpolated), so neighbouring cells share their faces exactly.
//
// Table per cell, in the point order of the psi tables (volume rule, then the
// six faces): J^{-1}[a][d] = d xi_a / d x_d (9 values) and a weight:
//   volume points: w |det J|;   face points: w_t1 w_t2 |det J| |J^{-T} e_D|.
#include "kern_common.h"

namespace dgwm {

namespace {

__device__ __forceinline__ double analytic_y(double x, double eta, double amp, double Lx) {
  const double yw = -1.0 + amp * cos(2.0 * M_PI * x / Lx);
  return yw + 0.5 * (eta + 1.0) * (1.0 - yw);
}

// Lagrange basis through `x` (n nodes) at t: values and derivatives.
__device__ void lagrange_at(const double* x, int n, double t, double* v, double* d) {
  for (int i = 0; i < n; ++i) {
    double p = 1.0, s = 0.0;
    for (int j = 0; j < n; ++j) {
      if (j == i) continue;
      p *= (t - x[j]) / (x[i] - x[j]);
    }
    for (int l = 0; l < n; ++l) {
      if (l == i) continue;
      double q = 1.0 / (x[i] - x[l]);
      for (int j = 0; j < n; ++j)
        if (j != i && j != l) q *= (t - x[j]) / (x[i] - x[j]);
      s += q;
    }
    v[i] = p;
    d[i] = s;
  }
}

// Reference coordinates and face/volume weight of point pt of a cell whose
// wall-normal rule has nqyc points.  Returns the face index (-1: volume).
template <int NQ>
__device__ int point_xi(int pt, int nqyc, const double* gq, const double* wq, const double* gyc,
                        const double* wyc, double xi[3], double& w) {
  const int npts = NQ * nqyc * NQ;
  if (pt < npts) {
    const int qx = pt % NQ, qy = (pt / NQ) % nqyc, qz = pt / (NQ * nqyc);
    xi[0] = gq[qx];
    xi[1] = gyc[qy];
    xi[2] = gq[qz];
    w = wq[qx] * wyc[qy] * wq[qz];
    return -1;
  }
  int f = 0, o = npts;
  while (pt >= o + psi_face_points(NQ, nqyc, f / 2)) {
    o += psi_face_points(NQ, nqyc, f / 2);
    ++f;
  }
  const int d = f / 2, s = f % 2, k = pt - o;
  const int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
  const int Q1 = t1 == 1 ? nqyc : NQ;
  const int q1 = k % Q1, q2 = k / Q1;
  xi[d] = (double)s;
  xi[t1] = t1 == 1 ? gyc[q1] : gq[q1];
  xi[t2] = t2 == 1 ? gyc[q2] : gq[q2];
  w = (t1 == 1 ? wyc[q1] : wq[q1]) * (t2 == 1 ? wyc[q2] : wq[q2]);
  return f;
}

template <int NP, int NQ, int NQY>
__global__ void geom_kernel(int nx, int ny, int nz, double Lx, double Lz, double amp, const double* __restrict__ eta,
                            const double* __restrict__ tab, int lower_slot, int upper_slot, int fully_periodic,
                            int stride, double* __restrict__ geo) {
  constexpr TabLayout L = tab_layout(NP, NQ, NQY);
  const int64_t ncell = (int64_t)nx * ny * nz;
  const int64_t gid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (gid >= ncell * stride) return;
  const int64_t e = gid / stride;
  const int pt = (int)(gid - e * stride);
  const int ex = (int)(e % nx), ey = (int)((e / nx) % ny);
  const bool enr = !fully_periodic && ((ey == 0 && lower_slot >= 0) || (ey == ny - 1 && upper_slot >= 0));
  const int nqyc = enr ? NQY : NQ;
  double* out = geo + gid * 10;
  if (pt >= psi_points(NQ, nqyc)) {
    for (int i = 0; i < 10; ++i) out[i] = 0.0;
    return;
  }
  double xi[3], w;
  const int f = point_xi<NQ>(pt, nqyc, tab + L.g, tab + L.w, enr ? tab + L.gy : tab + L.g,
                             enr ? tab + L.wy : tab + L.w, xi, w);
  const double hx = Lx / nx, hz = Lz / nz;
  const double x0 = ex * hx, e0 = eta[ey], he = eta[ey + 1] - eta[ey];
  const double* gl = tab + L.gl;
  double vx[NP], dx[NP], vy[NP], dy[NP];
  lagrange_at(gl, NP, xi[0], vx, dx);
  lagrange_at(gl, NP, xi[1], vy, dy);
  double yx = 0, yy = 0;
  for (int i = 0; i < NP; ++i)
    for (int j = 0; j < NP; ++j) {
      const double Y = analytic_y(x0 + hx * gl[i], e0 + he * gl[j], amp, Lx);
      yx += dx[i] * vy[j] * Y;
      yy += vx[i] * dy[j] * Y;
    }
  // J = [[hx, 0, 0], [yx, yy, 0], [0, 0, hz]]
  const double J[3][3] = {{hx, 0.0, 0.0}, {yx, yy, 0.0}, {0.0, 0.0, hz}};
  const double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                     J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
  double Ji[3][3];
  Ji[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) / det;
  Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
  Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
  Ji[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) / det;
  Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
  Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
  Ji[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) / det;
  Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
  Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
  for (int a = 0; a < 3; ++a)
    for (int d = 0; d < 3; ++d) out[3 * a + d] = Ji[a][d];
  double wt = w * fabs(det);
  if (f >= 0) {
    const int d = f / 2;
    wt *= sqrt(Ji[d][0] * Ji[d][0] + Ji[d][1] * Ji[d][1] + Ji[d][2] * Ji[d][2]);
  }
  out[9] = wt;
}

// Volume and the six face areas of each cell (fixed-order block sums).
template <int NQ, int NQY>
__global__ __launch_bounds__(64) void measure_kernel(int nx, int ny, int lower_slot, int upper_slot,
                                                     int fully_periodic, int stride, const double* __restrict__ geo,
                                                     double* __restrict__ meas /* [cell][7] */) {
  __shared__ double red[64];
  const int64_t e = blockIdx.x;
  const int ey = (int)((e / nx) % ny);
  const bool enr = !fully_periodic && ((ey == 0 && lower_slot >= 0) || (ey == ny - 1 && upper_slot >= 0));
  const int nqyc = enr ? NQY : NQ;
  const double* g = geo + e * stride * 10;
  for (int part = 0; part < 7; ++part) {
    const int lo = part == 0 ? 0 : psi_face_offset(NQ, nqyc, part - 1);
    const int hi = part == 0 ? NQ * nqyc * NQ : psi_face_offset(NQ, nqyc, part);
    double s = 0;
    for (int p = lo + (int)threadIdx.x; p < hi; p += 64) s += g[p * 10 + 9];
    red[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = 0;
      for (int i = 0; i < 64; ++i) t += red[i];
      meas[e * 7 + part] = t;
    }
    __syncthreads();
  }
}

// tau_F = pen (|F|/|Omega-| or, on walls, wall_mult |F|/|Omega-|, else the
// max over both cells), |F| from the cell's own face rule.
__global__ void tau_kernel(int nx, int ny, int nz, int fully_periodic, double pen, double wall_mult,
                           const double* __restrict__ meas, double* __restrict__ tauF) {
  const int64_t ncell = (int64_t)nx * ny * nz;
  const int64_t gid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (gid >= ncell * 6) return;
  const int64_t e = gid / 6;
  const int f = (int)(gid - e * 6), d = f / 2, s = f % 2;
  int n[3] = {(int)(e % nx), (int)((e / nx) % ny), (int)(e / ((int64_t)nx * ny))};
  const int nmax = d == 0 ? nx : (d == 1 ? ny : nz);
  int j = (d == 0 ? n[0] : (d == 1 ? n[1] : n[2])) + (s ? 1 : -1);
  const double area = meas[e * 7 + 1 + f], vol = meas[e * 7];
  if (j < 0 || j >= nmax) {
    if (d == 1 && !fully_periodic) {
      tauF[gid] = pen * wall_mult * area / vol;
      return;
    }
    j = (j + nmax) % nmax;
  }
  const int n0 = d == 0 ? j : n[0], n1 = d == 1 ? j : n[1], n2 = d == 2 ? j : n[2];
  const int64_t nb = n0 + (int64_t)nx * (n1 + (int64_t)ny * n2);
  tauF[gid] = pen * fmax(area / vol, area / meas[nb * 7]);
}

}  // namespace

#define DG_GEOM_COMBOS(X) X(3, 4, 8) X(3, 4, 4) X(4, 4, 8) X(4, 5, 8) X(4, 5, 5) X(5, 7, 8) X(6, 8, 8)

int launch_geometry(const dg_mesh* m, hipStream_t s) {
  const int64_t n = m->ncell * m->geo_stride;
  const unsigned nb = (unsigned)((n + 127) / 128);
  const int np = m->np_u, nq = m->P.nq_u, nqw = m->P.nq_wn;
#define X(a, b, c)                                                                                            \
  if (np == a && nq == b && nqw == c) {                                                                       \
    hipLaunchKernelGGL((geom_kernel<a, b, c>), dim3(nb), dim3(128), 0, s, m->P.nx, m->P.ny, m->P.nz, m->P.Lx, \
                       m->P.Lz, m->P.wall_amp, m->eta, m->tab_u, m->lower_slot, m->upper_slot,                \
                       m->P.fully_periodic, m->geo_stride, m->geo);                                           \
    hipLaunchKernelGGL((measure_kernel<b, c>), dim3((unsigned)m->ncell), dim3(64), 0, s, m->P.nx, m->P.ny,    \
                       m->lower_slot, m->upper_slot, m->P.fully_periodic, m->geo_stride, m->geo, m->meas);     \
    hipLaunchKernelGGL(tau_kernel, dim3((unsigned)((m->ncell * 6 + 255) / 256)), dim3(256), 0, s, m->P.nx,    \
                       m->P.ny, m->P.nz, m->P.fully_periodic,                                                 \
                       m->P.ip_factor_u * (m->P.k_u + 1.0) * (m->P.k_u + 1.0), m->P.wall_ip_mult, m->meas,    \
                       m->tauF);                                                                              \
    return check_hip(hipGetLastError(), "geometry kernels");                                                  \
  }
  DG_GEOM_COMBOS(X)
#undef X
  return set_error(DG_ERR_UNSUPPORTED, "curved geometry: degree/quadrature combination not compiled");
}

}  // namespace dgwm
