// Nodal wall shear stress of both walls (arXiv 1705.08813, Sec. 3.2), FP64.
//
//   tau_w,B = || int_wall N_B nu (grad u_h) n dA || / int_wall N_B dA
//
// N_B is the bilinear hat function of wall vertex B on the periodic
// (x, z) vertex grid of a wall, n the outward unit normal (-e_y on the lower
// wall, +e_y on the upper one) and u_h the full velocity, including psi u~ in
// enriched cells (psi sum_B N_B u~_B with l = 1).  On a flat wall (grad u) n = -+ du/dy, so only the
// wall-normal derivative at the wall-face Gauss points of the velocity rule
// is needed:
//   du_c/dy = (1/h_y) sum_B N_B'(wall) u_cB + u~_c dpsi/dy,
// the last term read from the stored psi table of the wall face.
//
// Two launches with a fixed summation order (deterministic):
//  1. one workgroup per wall cell: du/dy at the nq x nq face points by
//     sum factorisation (contract y with N'(0) or N'(1), then x and z with
//     the interpolation matrix), times nu n_y w_qx w_qz hx hz, then weighted
//     by the four corner hats; 12 numbers (4 corners x 3 components) per
//     cell go to the scratch array part[wall][ez][ex][corner][c].
//  2. one thread per wall vertex: the four adjacent cells' corner vectors
//     summed in a fixed order, the norm taken and divided by
//     int N_B dA = hx hz (the hat's area on a uniform periodic grid).
#include "kern_common.h"

namespace dgwm {

namespace {

constexpr int kWsThreads = 128;

// blockIdx.x = ex + nx (ez + nz w): the wall cell; part has 12 doubles per block.
__global__ __launch_bounds__(kWsThreads) void wall_shear_cells(
    int nx, int ny, int nz, int np, int nq, int nq_wn, const double* __restrict__ tab, const double* __restrict__ hy,
    double hx, double hz, double nu, int lower_slot, int upper_slot, int nslots, int64_t ncell, int psi_pts, int nle,
    const double* __restrict__ u, const double* __restrict__ psi, double* __restrict__ part) {
  __shared__ double sS[kMaxQ * kMaxP], sNd[kMaxP], sG[kMaxQ], sW[kMaxQ];
  __shared__ double v[3 * kMaxP * kMaxP];   // [c][k][i]  y contracted
  __shared__ double t[3 * kMaxP * kMaxQ];   // [c][k][qx] x interpolated
  __shared__ double f[3 * kMaxQ * kMaxQ];   // [c][qz][qx] weighted traction
  __shared__ double r[3 * kMaxQ * 2];       // [c][qz][a]  x hats applied
  const int tid = threadIdx.x;
  const int ex = blockIdx.x % nx;
  const int rest = blockIdx.x / nx;
  const int ez = rest % nz;
  const int w = rest / nz;
  const int ey = w ? ny - 1 : 0;
  const TabLayout L = tab_layout(np, nq, nq_wn);
  for (int i = tid; i < nq * np; i += kWsThreads) sS[i] = tab[L.S + i];
  if (tid < np) sNd[tid] = tab[(w ? L.nd1 : L.nd0) + tid];
  if (tid < nq) {
    sG[tid] = tab[L.g + tid];
    sW[tid] = tab[L.w + tid];
  }
  __syncthreads();
  const int np2 = np * np, np3 = np2 * np;
  const double* ue = u + (ex + (int64_t)nx * (ey + (int64_t)ny * ez)) * 3 * np3;
  // node B = i + np (j + np k): contract j with N_j'(wall)
  for (int it = tid; it < 3 * np2; it += kWsThreads) {
    const int c = it / np2, ki = it - c * np2, k = ki / np, i = ki - k * np;
    const double* p = ue + c * np3 + k * np2 + i;
    double s = 0.0;
    for (int j = 0; j < np; ++j) s += sNd[j] * p[j * np];
    v[it] = s;
  }
  __syncthreads();
  for (int it = tid; it < 3 * np * nq; it += kWsThreads) {
    const int ck = it / nq, qx = it - ck * nq;
    double s = 0.0;
    for (int i = 0; i < np; ++i) s += sS[qx * np + i] * v[ck * np + i];
    t[it] = s;
  }
  __syncthreads();
  const int slot = w ? upper_slot : lower_slot;
  const int64_t enr = slot < 0 ? -1 : ex + (int64_t)nx * (slot + (int64_t)nslots * ez);
  const double ihy = hy[ny + ey];
  const double scale = nu * (w ? 1.0 : -1.0) * hx * hz;  // nu n_y dA / (w_qx w_qz)
  const int nq2 = nq * nq;
  // psi face of the wall: y-face s = w, points qx + nq qz, entry 2 = dpsi/dy
  const double* pw = enr < 0 ? nullptr : psi + (enr * psi_pts + psi_face_offset(nq, nq_wn, 2 + w)) * 4 + 2;
  const double* ut = enr < 0 ? nullptr : u + ncell * 3 * np3 + enr * 3 * nle;
  for (int it = tid; it < 3 * nq2; it += kWsThreads) {
    const int c = it / nq2, q = it - c * nq2, qz = q / nq, qx = q - qz * nq;
    double s = 0.0;
    for (int k = 0; k < np; ++k) s += sS[qz * np + k] * t[(c * np + k) * nq + qx];
    double d = s * ihy;
    if (pw) {
      // psi vanishes on the wall: d/dy (psi sum_B N_B u~_B) = (sum_B N_B u~_B) dpsi/dy there, with only the
      // four vertex functions of the wall face (bit w along y) nonzero for l = 1
      double wt = ut[c * nle];
      if (nle == 8) {
        const double gx = sG[qx], gz = sG[qz];
        wt = 0.0;
        for (int j = 0; j < 4; ++j) {
          const int bx = j & 1, bz = j >> 1;
          wt += (bx ? gx : 1.0 - gx) * (bz ? gz : 1.0 - gz) * ut[c * 8 + (bx | (w << 1) | (bz << 2))];
        }
      }
      d += wt * pw[q * 4];
    }
    f[it] = scale * sW[qx] * sW[qz] * d;
  }
  __syncthreads();
  // x hats: N_0 = 1 - xi, N_1 = xi
  for (int it = tid; it < 3 * nq * 2; it += kWsThreads) {
    const int a = it & 1, cq = it >> 1;  // cq = c nq + qz
    const double* fr = f + cq * nq;
    double s = 0.0;
    for (int qx = 0; qx < nq; ++qx) s += (a ? sG[qx] : 1.0 - sG[qx]) * fr[qx];
    r[it] = s;
  }
  __syncthreads();
  // z hats; corner = 2 cz + a, output [corner][c]
  if (tid < 12) {
    const int corner = tid / 3, c = tid - corner * 3, cz = corner >> 1, a = corner & 1;
    double s = 0.0;
    for (int qz = 0; qz < nq; ++qz) s += (cz ? sG[qz] : 1.0 - sG[qz]) * r[(c * nq + qz) * 2 + a];
    part[(int64_t)blockIdx.x * 12 + tid] = s;
  }
}

// node = jx + nx (jz + nz w)
__global__ void wall_shear_nodes_kernel(int nx, int nz, double inv_area, const double* __restrict__ part,
                                        double* __restrict__ out) {
  const int64_t node = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (node >= 2 * (int64_t)nz * nx) return;
  const int jx = (int)(node % nx);
  const int64_t rest = node / nx;
  const int jz = (int)(rest % nz);
  const int w = (int)(rest / nz);
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
  for (int cz = 0; cz < 2; ++cz)
    for (int a = 0; a < 2; ++a) {
      const int ex = jx - a < 0 ? jx - a + nx : jx - a;
      const int ez = jz - cz < 0 ? jz - cz + nz : jz - cz;
      const double* p = part + (((int64_t)w * nz + ez) * nx + ex) * 12 + (2 * cz + a) * 3;
      s0 += p[0];
      s1 += p[1];
      s2 += p[2];
    }
  out[node] = sqrt(s0 * s0 + s1 * s1 + s2 * s2) * inv_area;
}

}  // namespace

int launch_wall_shear_nodes(const dg_mesh* m, const double* u, double* out, hipStream_t s) {
  const dg_mesh_params& P = m->P;
  if (m->np_u > kMaxP || P.nq_u > kMaxQ) return set_error(DG_ERR_UNSUPPORTED, "wall shear: degree too high");
  const int64_t ncellw = 2 * (int64_t)P.nz * P.nx;
  if (ncellw > INT32_MAX) return set_error(DG_ERR_ARG, "wall shear: too many wall cells");
  const double* tab = m->tab_u;
  hipLaunchKernelGGL(wall_shear_cells, dim3((unsigned)ncellw), dim3(kWsThreads), 0, s, P.nx, P.ny, P.nz, m->np_u,
                     P.nq_u, P.nq_wn, tab, m->hy, m->hx, m->hz, P.nu, m->lower_slot, m->upper_slot,
                     m->n_enr_layers, m->ncell, m->psi_pts, m->nle, u, m->psi, m->ws_part);
  int rc = check_hip(hipGetLastError(), "wall shear cell kernel launch");
  if (rc) return rc;
  hipLaunchKernelGGL(wall_shear_nodes_kernel, dim3((unsigned)((ncellw + 255) / 256)), dim3(256), 0, s, P.nx, P.nz,
                     1.0 / (m->hx * m->hz), m->ws_part, out);
  return check_hip(hipGetLastError(), "wall shear node kernel launch");
}

}  // namespace dgwm
