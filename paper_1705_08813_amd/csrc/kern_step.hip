// Vorticity and the high-order pressure Neumann data of the dual-splitting
// scheme (arXiv 1705.08813, Sec. 4.1 eq. bc_d_pres, Sec. 4.2 eq. ipflux on
// the walls), FP64, flat (box) meshes.
//
//   vorticity right-hand side  b(v) = (v, curl u)_e  for every velocity test
//     function (N_B e_c, and in enriched cells psi e_c for l = 0 or psi N_B e_c
//     over the eight trilinear vertex functions for l = 1, Sec. 3.1 eq.
//     enrichment), u = u_bar + psi sum_B N_B u~_B,
//     the cell's velocity rule; omega = M^{-1} b is the L2 projection of
//     curl u onto the enriched velocity space;
//   wall term  rhs(q) += int_wall q h_N dA,
//     h_N = -( sum_i beta_i (div(u_i (x) u_i) + nu curl omega_i) - f ) . n,
//     at the Gauss points of the velocity face rule, n = -e_y (lower wall),
//     +e_y (upper wall).
// Both are cell-local: one workgroup per cell (per wall cell), values and
// gradients at the points by direct sums over the cell's nodal basis (the
// points and basis functions of one cell fit in LDS and registers), then the
// test integrals.
#include "kern_common.h"

namespace dgwm {

namespace {

constexpr int kVortThreads = 256;

// Trilinear vertex function B (B = bx + 2 (by + 2 bz)) at reference point x
// and its physical gradient (ih: reciprocal cell sizes).
__device__ __forceinline__ double st_vtx(int B, const double x[3], const double ih[3], double g[3]) {
  const double a0 = (B & 1) ? x[0] : 1.0 - x[0], a1 = (B & 2) ? x[1] : 1.0 - x[1], a2 = (B & 4) ? x[2] : 1.0 - x[2];
  g[0] = ((B & 1) ? ih[0] : -ih[0]) * a1 * a2;
  g[1] = a0 * ((B & 2) ? ih[1] : -ih[1]) * a2;
  g[2] = a0 * a1 * ((B & 4) ? ih[2] : -ih[2]);
  return a0 * a1 * a2;
}

// Cell layout helpers: (ex, ey, ez) of cell e.
__device__ __forceinline__ void cell_xyz(const MeshDev& M, int e, int& ex, int& ey, int& ez) {
  ex = e % M.nx;
  const int t = e / M.nx;
  ey = t % M.ny;
  ez = t / M.ny;
}

// b(v) = (v, curl u)_e on the cells of one class (ENR: enriched cells with the
// NQY-point wall-normal rule; else the others, NQY = NQ).  One block per cell;
// blocks of the other class leave at once.
template <int NP, int NQ, int NQY, bool ENR, int LE = 1>
__global__ __launch_bounds__(kVortThreads) void vort_rhs_kernel(const MeshDev M, const double* __restrict__ u,
                                                                double* __restrict__ b) {
  constexpr int NP3 = NP * NP * NP, NPT = NQ * NQY * NQ;
  constexpr TabLayout L = tab_layout(NP, NQ, NQY);
  __shared__ double sU[3 * NP3];
  __shared__ double sCW[3 * NPT];  // [component][point]: w |J| curl u
  __shared__ double sPsi[ENR ? NPT : 1];
  __shared__ double sUt[ENR ? 3 * LE : 1];  // the cell's enrichment coefficients [c][B]
  const int e = blockIdx.x;
  int ex, ey, ez;
  cell_xyz(M, e, ex, ey, ez);
  const int64_t k = enr_index(M, ex, ey, ez);
  if (ENR != (k >= 0)) return;  // uniform over the block, before any barrier
  const double hx = M.hx, hy = M.hy[ey], hz = M.hz;
  const double vol = hx * hy * hz;
  for (int t = threadIdx.x; t < 3 * NP3; t += blockDim.x) sU[t] = u[(int64_t)e * 3 * NP3 + t];
  if (ENR && threadIdx.x < 3 * LE) sUt[threadIdx.x] = u[M.enr_off + 3 * LE * k + threadIdx.x];
  __syncthreads();
  const double* tab = M.tab;
  const double* Sx = tab + L.S;
  const double* Dx = tab + L.Sd;
  const double* Sy = tab + (ENR ? L.Sy : L.S);
  const double* Dy = tab + (ENR ? L.Sdy : L.Sd);
  const double* wq = tab + L.w;
  const double* wy = tab + (ENR ? L.wy : L.w);
  for (int t = threadIdx.x; t < NPT; t += blockDim.x) {
    const int qx = t % NQ, qy = (t / NQ) % NQY, qz = t / (NQ * NQY);
    double g[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};  // [component][direction]
    for (int m = 0; m < NP; ++m) {
      const double vz = Sx[qz * NP + m], dz = Dx[qz * NP + m];
      for (int j = 0; j < NP; ++j) {
        const double vy = Sy[qy * NP + j], dy = Dy[qy * NP + j];
#pragma unroll
        for (int i = 0; i < NP; ++i) {
          const double vx = Sx[qx * NP + i], dx = Dx[qx * NP + i];
          const double nx = dx * vy * vz, ny = vx * dy * vz, nz = vx * vy * dz;
          const int B = i + NP * (j + NP * m);
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            const double uc = sU[c * NP3 + B];
            g[c][0] += uc * nx;
            g[c][1] += uc * ny;
            g[c][2] += uc * nz;
          }
        }
      }
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      g[c][0] /= hx;
      g[c][1] /= hy;
      g[c][2] /= hz;
    }
    if (ENR) {
      const double* p4 = M.psi + ((int64_t)k * M.psi_pts + M.psi_off[0] + t) * 4;
      if (LE == 1) {
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
          for (int d = 0; d < 3; ++d) g[c][d] += sUt[c] * p4[1 + d];
      } else {
        // grad(psi sum_B N_B ut_B) = sum_B ut_B (N_B grad psi + psi grad N_B)
        const double x[3] = {tab[L.g + qx], tab[L.gy + qy], tab[L.g + qz]}, ih[3] = {1.0 / hx, 1.0 / hy, 1.0 / hz};
#pragma unroll
        for (int B = 0; B < 8; ++B) {
          double gn[3];
          const double nb = st_vtx(B, x, ih, gn);
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            const double w = sUt[c * LE + B];
#pragma unroll
            for (int d = 0; d < 3; ++d) g[c][d] += w * (nb * p4[1 + d] + p4[0] * gn[d]);
          }
        }
      }
      sPsi[t] = p4[0];
    }
    const double w = wq[qx] * wy[qy] * wq[qz] * vol;
    sCW[0 * NPT + t] = w * (g[2][1] - g[1][2]);
    sCW[1 * NPT + t] = w * (g[0][2] - g[2][0]);
    sCW[2 * NPT + t] = w * (g[1][0] - g[0][1]);
  }
  __syncthreads();
  for (int t = threadIdx.x; t < 3 * NP3; t += blockDim.x) {
    const int c = t / NP3, B = t % NP3;
    const int i = B % NP, j = (B / NP) % NP, m = B / (NP * NP);
    const double* cw = sCW + c * NPT;
    double s = 0;
    for (int qz = 0; qz < NQ; ++qz) {
      const double vz = Sx[qz * NP + m];
      for (int qy = 0; qy < NQY; ++qy) {
        const double vyz = Sy[qy * NP + j] * vz;
        const double* row = cw + NQ * (qy + NQY * qz);
#pragma unroll
        for (int qx = 0; qx < NQ; ++qx) s += Sx[qx * NP + i] * vyz * row[qx];
      }
    }
    b[(int64_t)e * 3 * NP3 + t] = s;
  }
  if (ENR && threadIdx.x < 3 * LE) {
    // enrichment rows: sum over the points of psi N_B w |J| curl u (N_B = 1 for l = 0)
    const int c = threadIdx.x / LE, B = threadIdx.x - c * LE;
    double s = 0;
    for (int q = 0; q < NPT; ++q) {
      double nb = 1.0;
      if (LE == 8) {
        const int qx = q % NQ, qy = (q / NQ) % NQY, qz = q / (NQ * NQY);
        const double x[3] = {tab[L.g + qx], tab[L.gy + qy], tab[L.g + qz]}, ih[3] = {1.0, 1.0, 1.0};
        double gn[3];
        nb = st_vtx(B, x, ih, gn);
      }
      s += sPsi[q] * nb * sCW[c * NPT + q];
    }
    b[M.enr_off + 3 * LE * k + threadIdx.x] = s;
  }
}

struct NeuArgs {
  const double* u[2];
  const double* om[2];
  double beta[2];
  int nh;
  double fy;           // body force, y component
  const double* glp;   // pressure Gauss-Lobatto nodes (npp)
  int npp;
};

// Wall term of the pressure equation: one block per wall cell (lower walls
// first), threads over the face points, then over the wall-layer pressure
// nodes of the cell (the other pressure basis functions vanish on the wall).
template <int NP, int NQ, int LE = 1>
__global__ __launch_bounds__(64) void neumann_kernel(const MeshDev M, const NeuArgs A, double* __restrict__ rhs) {
  constexpr int NP3 = NP * NP * NP, NF = NQ * NQ;
  constexpr TabLayout L = tab_layout(NP, NQ, NQ);  // (the S, Sd, w, g, nd tables precede the y rule)
  __shared__ double sH[NF];
  const int wall = blockIdx.x / (M.nx * M.nz);
  const int r = blockIdx.x % (M.nx * M.nz);
  const int ex = r % M.nx, ez = r / M.nx;
  const int ey = wall ? M.ny - 1 : 0;
  const double sg = wall ? 1.0 : -1.0;  // outward normal sg e_y
  const int e = ex + M.nx * (ey + M.ny * ez);
  const int64_t k = enr_index(M, ex, ey, ez);
  const double hx = M.hx, hy = M.hy[ey], hz = M.hz;
  const double* tab = M.tab;
  const double* S = tab + L.S;
  const double* D = tab + L.Sd;
  const double* wq = tab + L.w;
  const double* nd = tab + (wall ? L.nd1 : L.nd0);
  const int jw = wall ? NP - 1 : 0;  // the node layer on the wall (the only one with N_j != 0 there)
  for (int t = threadIdx.x; t < NF; t += blockDim.x) {
    const int qx = t % NQ, qz = t / NQ;
    const double* p4 = k >= 0 ? M.psi + ((int64_t)k * M.psi_pts + M.psi_off[1 + (wall ? 3 : 2)] + t) * 4 : nullptr;
    double hn = 0;
    for (int h = 0; h < A.nh; ++h) {
      const double* ue = A.u[h] + (int64_t)e * 3 * NP3;
      const double* oe = A.om[h] + (int64_t)e * 3 * NP3;
      double val[3] = {0, 0, 0}, g[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}}, gox_z = 0, goz_x = 0;
      for (int m = 0; m < NP; ++m) {
        const double vz = S[qz * NP + m], dz = D[qz * NP + m] / hz;
        for (int j = 0; j < NP; ++j) {
          const double vy = j == jw ? 1.0 : 0.0, dy = nd[j] / hy;
#pragma unroll
          for (int i = 0; i < NP; ++i) {
            const double vx = S[qx * NP + i], dx = D[qx * NP + i] / hx;
            const int B = i + NP * (j + NP * m);
            const double n0 = vx * vy * vz, nxd = dx * vy * vz, nyd = vx * dy * vz, nzd = vx * vy * dz;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
              const double uc = ue[c * NP3 + B];
              val[c] += uc * n0;
              g[c][0] += uc * nxd;
              g[c][1] += uc * nyd;
              g[c][2] += uc * nzd;
            }
            gox_z += oe[0 * NP3 + B] * nzd;
            goz_x += oe[2 * NP3 + B] * nxd;
          }
        }
      }
      if (p4) {
        const double* ut = A.u[h] + M.enr_off + 3 * LE * k;
        const double* ot = A.om[h] + M.enr_off + 3 * LE * k;
        if (LE == 1) {
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            val[c] += ut[c] * p4[0];
#pragma unroll
            for (int d = 0; d < 3; ++d) g[c][d] += ut[c] * p4[1 + d];
          }
          gox_z += ot[0] * p4[3];
          goz_x += ot[2] * p4[1];
        } else {
          // enrichment psi sum_B N_B ut_B and its gradient sum_B ut_B (N_B grad psi + psi grad N_B) at the wall
          // point (psi vanishes there, its gradient does not)
          const double x[3] = {tab[L.g + qx], wall ? 1.0 : 0.0, tab[L.g + qz]}, ih[3] = {1.0 / hx, 1.0 / hy, 1.0 / hz};
#pragma unroll
          for (int B = 0; B < 8; ++B) {
            double gn[3];
            const double nb = st_vtx(B, x, ih, gn);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
              val[c] += ut[c * LE + B] * nb * p4[0];
#pragma unroll
              for (int d = 0; d < 3; ++d) g[c][d] += ut[c * LE + B] * (nb * p4[1 + d] + p4[0] * gn[d]);
            }
            gox_z += ot[0 * LE + B] * (nb * p4[3] + p4[0] * gn[2]);
            goz_x += ot[2 * LE + B] * (nb * p4[1] + p4[0] * gn[0]);
          }
        }
      }
      const double div = g[0][0] + g[1][1] + g[2][2];
      const double conv_y = g[1][0] * val[0] + g[1][1] * val[1] + g[1][2] * val[2] + val[1] * div;
      const double curl_y = gox_z - goz_x;
      hn += A.beta[h] * sg * (conv_y + M.nu * curl_y);
    }
    hn = -hn + sg * A.fy;
    sH[t] = hn * wq[qx] * wq[qz] * hx * hz;
  }
  __syncthreads();
  // pressure basis at the velocity Gauss points of x and z (Lagrange form)
  const int npp = A.npp;
  const double* g1 = tab + L.g;
  for (int t = threadIdx.x; t < npp * npp; t += blockDim.x) {
    const int i = t % npp, m = t / npp;
    double s = 0;
    for (int qz = 0; qz < NQ; ++qz) {
      double lz = 1.0;
      for (int a = 0; a < npp; ++a)
        if (a != m) lz *= (g1[qz] - A.glp[a]) / (A.glp[m] - A.glp[a]);
      for (int qx = 0; qx < NQ; ++qx) {
        double lx = 1.0;
        for (int a = 0; a < npp; ++a)
          if (a != i) lx *= (g1[qx] - A.glp[a]) / (A.glp[i] - A.glp[a]);
        s += lx * lz * sH[qx + NQ * qz];
      }
    }
    const int j = wall ? npp - 1 : 0;
    const int64_t o = (int64_t)e * npp * npp * npp + i + npp * (j + npp * m);
    rhs[o] += s;
  }
}

MeshDev step_meshdev(const dg_mesh* m) {
  MeshDev M{};
  M.nx = m->P.nx;
  M.ny = m->P.ny;
  M.nz = m->P.nz;
  M.fully_periodic = m->P.fully_periodic;
  M.lower_slot = m->lower_slot;
  M.upper_slot = m->upper_slot;
  M.nslots = m->n_enr_layers;
  M.hx = m->hx;
  M.hz = m->hz;
  M.hy = m->hy;
  M.ihy = m->hy + m->P.ny;
  M.ihx = 1.0 / m->hx;
  M.ihz = 1.0 / m->hz;
  M.tab = m->tab_u;
  M.psi = m->psi;
  M.psi_pts = m->psi_pts;
  for (int f = 0; f <= 6; ++f) M.psi_off[f] = (f == 0) ? 0 : psi_face_offset(m->P.nq_u, m->P.nq_wn, f - 1);
  M.nu = m->P.nu;
  M.enr_off = m->ncell * 3 * (int64_t)m->np_u * m->np_u * m->np_u;
  M.nq_wn = m->P.nq_wn;
  return M;
}

}  // namespace

// (np, nq, nq_wn) combinations, as for the velocity residual
#define DG_STEP_COMBOS(X) X(3, 4, 8) X(3, 4, 4) X(4, 4, 8) X(4, 5, 8) X(4, 5, 5) X(5, 7, 8) X(6, 8, 8)

int launch_vorticity_rhs(const dg_mesh* m, const double* u, double* b, hipStream_t s) {
  if (m->curved) return launch_vorticity_rhs_curved(m, u, b, s);
  const MeshDev M = step_meshdev(m);
  const int np = m->np_u, nq = m->P.nq_u, nqw = m->P.nq_wn;
  const unsigned g = (unsigned)m->ncell;
  bool done = false;
#define X(a, q, w)                                                                                       \
  if (!done && np == a && nq == q && (nqw == w || m->nenr == 0)) {                                       \
    done = true;                                                                                         \
    hipLaunchKernelGGL((vort_rhs_kernel<a, q, q, false>), dim3(g), dim3(kVortThreads), 0, s, M, u, b);  \
    if (m->nenr > 0 && m->nle == 8)                                                                      \
      hipLaunchKernelGGL((vort_rhs_kernel<a, q, w, true, 8>), dim3(g), dim3(kVortThreads), 0, s, M, u, b); \
    else if (m->nenr > 0)                                                                                \
      hipLaunchKernelGGL((vort_rhs_kernel<a, q, w, true>), dim3(g), dim3(kVortThreads), 0, s, M, u, b); \
  }
  DG_STEP_COMBOS(X)
#undef X
  if (!done) return set_error(DG_ERR_UNSUPPORTED, "velocity degree/quadrature combination not compiled");
  return check_hip(hipGetLastError(), "vorticity launch");
}

int launch_pressure_neumann(const dg_mesh* m, int nh, const double* const* us, const double* const* oms,
                            const double* beta, const double* f, double* rhs, hipStream_t s) {
  if (m->P.fully_periodic) return DG_OK;  // no walls
  const MeshDev M = step_meshdev(m);
  NeuArgs A{};
  for (int h = 0; h < nh; ++h) {
    A.u[h] = us[h];
    A.om[h] = oms[h];
    A.beta[h] = beta[h];
  }
  A.nh = nh;
  A.fy = f ? f[1] : 0.0;
  A.glp = m->tab_p + tab_layout(m->np_p, m->P.nq_p, m->P.nq_p).gl;
  A.npp = m->np_p;
  const unsigned g = (unsigned)(2 * m->P.nx * m->P.nz);
  const int np = m->np_u, nq = m->P.nq_u;
  bool done = false;
#define X(a, q, w)                                                                                  \
  if (!done && np == a && nq == q) {                                                                \
    done = true;                                                                                    \
    if (m->nle == 8)                                                                                \
      hipLaunchKernelGGL((neumann_kernel<a, q, 8>), dim3(g), dim3(64), 0, s, M, A, rhs);            \
    else                                                                                            \
      hipLaunchKernelGGL((neumann_kernel<a, q>), dim3(g), dim3(64), 0, s, M, A, rhs);               \
  }
  DG_STEP_COMBOS(X)
#undef X
  if (!done) return set_error(DG_ERR_UNSUPPORTED, "velocity degree/quadrature combination not compiled");
  return check_hip(hipGetLastError(), "pressure Neumann launch");
}

}  // namespace dgwm

using namespace dgwm;

extern "C" {

int dg_vorticity_rhs(const dg_mesh* m, const double* u, double* b, void* stream) {
  if (!m || !u || !b) return set_error(DG_ERR_ARG, "mesh/u/b is NULL");
  if (u == b) return set_error(DG_ERR_ARG, "u and b must not alias");
  return launch_vorticity_rhs(m, u, b, static_cast<hipStream_t>(stream));
}

int dg_vorticity(const dg_mesh* m, const double* u, double* omega, void* stream) {
  if (!m || !u || !omega) return set_error(DG_ERR_ARG, "mesh/u/omega is NULL");
  if (u == omega) return set_error(DG_ERR_ARG, "u and omega must not alias");
  const hipStream_t s = static_cast<hipStream_t>(stream);
  int rc = launch_vorticity_rhs(m, u, omega, s);
  if (!rc) rc = launch_inverse_mass(m, omega, omega, s);
  return rc;
}

int dg_pressure_neumann(const dg_mesh* m, int32_t nhist, const double* const* u, const double* const* omega,
                        const double* beta, const double* f, double* rhs, void* stream) {
  if (!m || !u || !omega || !beta || !rhs) return set_error(DG_ERR_ARG, "mesh/u/omega/beta/rhs is NULL");
  if (nhist < 1 || nhist > 2) return set_error(DG_ERR_ARG, "nhist must be 1 or 2");
  for (int h = 0; h < nhist; ++h)
    if (!u[h] || !omega[h]) return set_error(DG_ERR_ARG, "a velocity or vorticity vector is NULL");
  if (m->curved)
    return launch_pressure_neumann_curved(m, nhist, u, omega, beta, f, rhs, static_cast<hipStream_t>(stream));
  return launch_pressure_neumann(m, nhist, u, omega, beta, f, rhs, static_cast<hipStream_t>(stream));
}

}  // extern "C"
