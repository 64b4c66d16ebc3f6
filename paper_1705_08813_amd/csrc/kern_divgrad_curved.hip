// Pressure gradient and velocity divergence terms of the dual-splitting
// scheme (arXiv 1705.08813, Sec. 4.2), the div-div penalty of its
// projection step, the inverse velocity mass matrix, the right-hand side of
// the projected vorticity and the pressure Neumann wall term on the
// curved-wall mesh, FP64:
//
//   P: g(v) = -(div v, p)_e + (v . n, {{p}})_{boundary of e}     (velocity test functions)
//   C: c(q) = -(grad q, u)_e + (q, {{u}} . n)_{boundary of e}    (pressure test functions)
//
// with the interior values on the no-slip walls, the full velocity (psi u~
// in enriched cells, l = 0) and the enrichment test functions psi e_c, as on
// flat meshes.  Every cell is mapped isoparametrically, so the geometry
// enters point by point from the mesh's geometry table (J^{-1} and the
// weight w |det J| at the volume points; w |det J| |J^{-T} e_d| at the face
// points, the outward normal being +-J^{-T} e_d normalised): with
// d_c N = sum_a J^{-1}[a][c] d_a N,
//
//   P volume:  g(N_B e_c) -= sum_q sum_a d_a N_B(q) F_ac(q),  F_ac = w|J| J^{-1}[a][c] p(q),
//   C volume:  c(N^p_B)   -= sum_q sum_a d_a N^p_B(q) F_a(q), F_a = w|J| sum_d J^{-1}[a][d] u_d(q),
//
// and the face terms integrate the face-layer basis functions (the
// Gauss-Lobatto nodal basis has its face values on that layer) against
// w dA n {{p}} or w dA {{u}} . n at the face points.  One workgroup per cell
// with the cell's block accumulated in LDS and written once; the 1-D tables
// of both bases at both rules are compile-time constants.  The volume terms
// of P and C interpolate and integrate by 1-D sweeps; the face terms and the
// other curved kernels use direct sums over the points (the curved
// configuration's hot path is the velocity operator).
#include "ctab.h"
#include "kern_common.h"

namespace dgwm {

namespace {

constexpr int kCvThreads = 256;

struct CvArgs {
  int nx, ny, nz, lower_slot, upper_slot, nslots, psi_pts, geo_stride, fully_periodic;
  int64_t ncell;
  const double* geo;  // [cell][geo_stride][J^{-1} (9), weight]
  const double* psi;  // [enr][psi_pts][4]: psi, grad psi (physical)
  const double* in;   // p (gradient) or u (divergence)
  double* out;
};

struct CvCell {
  int i[3];
  int64_t e, enr;
};

__device__ __forceinline__ int64_t cv_enr(const CvArgs& A, int ex, int ey, int ez) {
  if (A.fully_periodic) return -1;
  int slot = -1;
  if (ey == 0 && A.lower_slot >= 0) slot = A.lower_slot;
  else if (ey == A.ny - 1 && A.upper_slot >= 0) slot = A.upper_slot;
  return slot < 0 ? -1 : ex + (int64_t)A.nx * (slot + (int64_t)A.nslots * ez);
}

// Regular cells: b = ex + nx (ly + nlayers ez), ey = layer_lo + ly; enriched
// cells: b = enriched index.
template <bool ENR>
__device__ __forceinline__ CvCell cv_cell(const CvArgs& A, int64_t b, int layer_lo, int nlayers) {
  CvCell c;
  c.i[0] = (int)(b % A.nx);
  const int64_t t0 = b / A.nx;
  if (ENR) {
    const int slot = (int)(t0 % A.nslots);
    c.i[2] = (int)(t0 / A.nslots);
    c.i[1] = slot == A.lower_slot ? 0 : A.ny - 1;
  } else {
    c.i[1] = layer_lo + (int)(t0 % nlayers);
    c.i[2] = (int)(t0 / nlayers);
  }
  c.e = c.i[0] + (int64_t)A.nx * (c.i[1] + (int64_t)A.ny * c.i[2]);
  c.enr = ENR ? b : -1;
  return c;
}

// Neighbour across face (d, s) and its enriched index (-1: none); -1 on a wall.
__device__ __forceinline__ int64_t cv_neighbour(const CvArgs& A, const CvCell& c, int d, int s, int64_t& nenr) {
  int i[3] = {c.i[0], c.i[1], c.i[2]};
  const int n[3] = {A.nx, A.ny, A.nz};
  int j = i[d] + (s ? 1 : -1);
  nenr = -1;
  if (j < 0 || j >= n[d]) {
    if (d == 1 && !A.fully_periodic) return -1;
    j = j < 0 ? j + n[d] : j - n[d];
  }
  i[d] = j;
  nenr = cv_enr(A, i[0], i[1], i[2]);
  return i[0] + (int64_t)A.nx * (i[1] + (int64_t)A.ny * i[2]);
}

// Node of position (l1, l2) on the layer of face (d, s) of an NP^3 block.
template <int NP>
__device__ __forceinline__ int cv_layer(int d, int s, int l1, int l2) {
  const int ld = s ? NP - 1 : 0;
  if (d == 0) return ld + NP * (l1 + NP * l2);
  if (d == 1) return l1 + NP * (ld + NP * l2);
  return l1 + NP * (l2 + NP * ld);
}

// Fixed-order block sum of NV values per thread.
template <int NV>
__device__ __forceinline__ void cv_block_sum(double (&v)[NV], double* red, int tid) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1)
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] += __shfl_down(v[k], off, 64);
  constexpr int NW = kCvThreads / 64;
  __syncthreads();
  if ((tid & 63) == 0)
#pragma unroll
    for (int k = 0; k < NV; ++k) red[k * NW + (tid >> 6)] = v[k];
  __syncthreads();
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    v[k] = 0.0;
    for (int w = 0; w < NW; ++w) v[k] += red[k * NW + w];
  }
}

// Tensor sweeps over NV nodal fields of NP^3 (vector stride NP^3): values at
// the NQ x QY x NQ points, and the transposed gradient integrals
//   Y[r][B] = sum_q sum_a d_a N_B(q) F[r][a][q]   (F: [NV][3][NPT]),
// each as 1-D sweeps x, y, z; X1 (NV NP^2 NQ) and X2 (NV NP QY NQ) are scratch.
template <int NP, int NQ, int QY, int NV, int D = -1>  // D >= 0: the derivative d/dxi_D instead of values
__device__ __forceinline__ void cv_interp(const double* P, double* T, double* X1, double* X2, int tid) {
  constexpr int NP3 = NP * NP * NP, NPT = NQ * QY * NQ, S1 = NP * NP * NQ, S2 = NP * QY * NQ;
  constexpr auto& tx = ct::tab<NP, NQ>;
  constexpr auto& ty = ct::tab<NP, QY>;
  for (int it = tid; it < NV * S1; it += kCvThreads) {
    const int r = it / S1, t = it - r * S1, qx = t % NQ, jk = t / NQ;
    double v = 0.0;
    for (int i = 0; i < NP; ++i) v += (D == 0 ? tx.Sd[qx][i] : tx.S[qx][i]) * P[r * NP3 + i + NP * jk];
    X1[it] = v;
  }
  __syncthreads();
  for (int it = tid; it < NV * S2; it += kCvThreads) {
    const int r = it / S2, t = it - r * S2, qx = t % NQ, qy = (t / NQ) % QY, k = t / (NQ * QY);
    double v = 0.0;
    for (int j = 0; j < NP; ++j) v += (D == 1 ? ty.Sd[qy][j] : ty.S[qy][j]) * X1[r * S1 + qx + NQ * (j + NP * k)];
    X2[it] = v;
  }
  __syncthreads();
  for (int it = tid; it < NV * NPT; it += kCvThreads) {
    const int r = it / NPT, q = it - r * NPT, qxy = q % (NQ * QY), qz = q / (NQ * QY);
    double v = 0.0;
    for (int k = 0; k < NP; ++k) v += (D == 2 ? tx.Sd[qz][k] : tx.S[qz][k]) * X2[r * S2 + qxy + NQ * QY * k];
    T[it] = v;
  }
  __syncthreads();
}

template <int NP, int NQ, int QY, int NV>
__device__ __forceinline__ void cv_project_grad(const double* F, double* Y, double* X1, double* X2, int tid) {
  constexpr int NP3 = NP * NP * NP, NPT = NQ * QY * NQ, S1 = NP * NP * NQ, S2 = NP * QY * NQ;
  constexpr auto& tx = ct::tab<NP, NQ>;
  constexpr auto& ty = ct::tab<NP, QY>;
  for (int a = 0; a < 3; ++a) {
    for (int it = tid; it < NV * S2; it += kCvThreads) {
      const int r = it / S2, t = it - r * S2, i = t % NP, qyz = t / NP;
      const double* f = F + (r * 3 + a) * NPT + NQ * qyz;
      double v = 0.0;
      for (int qx = 0; qx < NQ; ++qx) v += (a == 0 ? tx.Sd[qx][i] : tx.S[qx][i]) * f[qx];
      X2[it] = v;
    }
    __syncthreads();
    for (int it = tid; it < NV * S1; it += kCvThreads) {
      const int r = it / S1, t = it - r * S1, i = t % NP, j = (t / NP) % NP, qz = t / (NP * NP);
      double v = 0.0;
      for (int qy = 0; qy < QY; ++qy) v += (a == 1 ? ty.Sd[qy][j] : ty.S[qy][j]) * X2[r * S2 + i + NP * (qy + QY * qz)];
      X1[it] = v;
    }
    __syncthreads();
    for (int it = tid; it < NV * NP3; it += kCvThreads) {
      const int r = it / NP3, B = it - r * NP3, ij = B % (NP * NP), k = B / (NP * NP);
      double v = 0.0;
      for (int qz = 0; qz < NQ; ++qz) v += (a == 2 ? tx.Sd[qz][k] : tx.S[qz][k]) * X1[r * S1 + ij + NP * NP * qz];
      Y[it] = a == 0 ? v : Y[it] + v;
    }
    __syncthreads();
  }
}

// Y[r][B] = sum_q N_B(q) F[r][q] (F: [NV][NPT]) by the transposed sweeps x, y, z.
template <int NP, int NQ, int QY, int NV>
__device__ __forceinline__ void cv_project_vals(const double* F, double* Y, double* X1, double* X2, int tid) {
  constexpr int NP3 = NP * NP * NP, NPT = NQ * QY * NQ, S1 = NP * NP * NQ, S2 = NP * QY * NQ;
  constexpr auto& tx = ct::tab<NP, NQ>;
  constexpr auto& ty = ct::tab<NP, QY>;
  for (int it = tid; it < NV * S2; it += kCvThreads) {
    const int r = it / S2, t = it - r * S2, i = t % NP, qyz = t / NP;
    const double* f = F + r * NPT + NQ * qyz;
    double v = 0.0;
    for (int qx = 0; qx < NQ; ++qx) v += tx.S[qx][i] * f[qx];
    X2[it] = v;
  }
  __syncthreads();
  for (int it = tid; it < NV * S1; it += kCvThreads) {
    const int r = it / S1, t = it - r * S1, i = t % NP, j = (t / NP) % NP, qz = t / (NP * NP);
    double v = 0.0;
    for (int qy = 0; qy < QY; ++qy) v += ty.S[qy][j] * X2[r * S2 + i + NP * (qy + QY * qz)];
    X1[it] = v;
  }
  __syncthreads();
  for (int it = tid; it < NV * NP3; it += kCvThreads) {
    const int r = it / NP3, B = it - r * NP3, ij = B % (NP * NP), k = B / (NP * NP);
    double v = 0.0;
    for (int qz = 0; qz < NQ; ++qz) v += tx.S[qz][k] * X1[r * S1 + ij + NP * NP * qz];
    Y[it] = v;
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// P: g = P p (velocity layout).
template <int NPU, int NPP, int NQ, int NQY, bool ENR>
__global__ __launch_bounds__(kCvThreads) void curved_gradient_kernel(const CvArgs A, int layer_lo, int nlayers) {
  constexpr int QY = ENR ? NQY : NQ;  // the cell's wall-normal rule
  constexpr int NU3 = NPU * NPU * NPU, NP3 = NPP * NPP * NPP, NPT = NQ * QY * NQ;
  constexpr int FMAX = NQ * (QY > NQ ? QY : NQ);
  constexpr auto& ux = ct::tab<NPU, NQ>;
  constexpr auto& uy = ct::tab<NPU, QY>;
  constexpr auto& px = ct::tab<NPP, NQ>;
  constexpr auto& py = ct::tab<NPP, QY>;
  __shared__ double sp[NP3];
  __shared__ double snb[6][NPP * NPP];
  __shared__ double F[3][3][NPT];  // [c][a]: w|J| J^{-1}[a][c] p
  __shared__ double pq[NPT];
  __shared__ double X1[3 * NPU * NPU * NQ], X2[3 * NPU * QY * NQ];
  __shared__ double G[3][FMAX];
  __shared__ double acc[3 * NU3];
  __shared__ double red[3 * (kCvThreads / 64)];
  __shared__ int64_t nbs[6];
  const int tid = threadIdx.x;
  const CvCell c = cv_cell<ENR>(A, blockIdx.x, layer_lo, nlayers);
  if (tid < 6) {
    int64_t ne;
    nbs[tid] = cv_neighbour(A, c, tid / 2, tid % 2, ne);
  }
  for (int k = tid; k < NP3; k += kCvThreads) sp[k] = A.in[c.e * NP3 + k];
  __syncthreads();
  for (int k = tid; k < 6 * NPP * NPP; k += kCvThreads) {
    const int f = k / (NPP * NPP), l = k - f * NPP * NPP;
    const int64_t nb = nbs[f];
    // the neighbour's layer on the shared face is its face (d, 1 - s)
    snb[f][l] = nb >= 0 ? A.in[nb * NP3 + cv_layer<NPP>(f / 2, 1 - f % 2, l % NPP, l / NPP)] : 0.0;
  }
  const double* geo = A.geo + c.e * (int64_t)A.geo_stride * 10;
  const double* ps = ENR ? A.psi + c.enr * (int64_t)A.psi_pts * 4 : nullptr;
  double ev[3] = {0.0, 0.0, 0.0};  // enrichment rows (thread partials)
  cv_interp<NPP, NQ, QY, 1>(sp, pq, X1, X2, tid);
  for (int q = tid; q < NPT; q += kCvThreads) {
    const double* g = geo + q * 10;
    const double v = pq[q], wv = g[9] * v;
#pragma unroll
    for (int cc = 0; cc < 3; ++cc)
#pragma unroll
      for (int a = 0; a < 3; ++a) F[cc][a][q] = wv * g[3 * a + cc];
    if (ENR)
#pragma unroll
      for (int cc = 0; cc < 3; ++cc) ev[cc] -= g[9] * ps[q * 4 + 1 + cc] * v;
  }
  __syncthreads();
  cv_project_grad<NPU, NQ, QY, 3>(&F[0][0][0], acc, X1, X2, tid);
  for (int it = tid; it < 3 * NU3; it += kCvThreads) acc[it] = -acc[it];
  __syncthreads();
  for (int f = 0; f < 6; ++f) {
    const int d = f / 2, s = f % 2;
    const int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
    const int Q1 = t1 == 1 ? QY : NQ, Q2 = t2 == 1 ? QY : NQ;
    const int off = psi_face_offset(NQ, QY, f);
    const bool wall = nbs[f] < 0;
    for (int k = tid; k < Q1 * Q2; k += kCvThreads) {
      const int q1 = k % Q1, q2 = k / Q1;
      double pm = 0.0, pp = 0.0;
      for (int l2 = 0; l2 < NPP; ++l2) {
        const double b2 = t2 == 1 ? py.S[q2][l2] : px.S[q2][l2];
        for (int l1 = 0; l1 < NPP; ++l1) {
          const double b = (t1 == 1 ? py.S[q1][l1] : px.S[q1][l1]) * b2;
          pm += b * sp[cv_layer<NPP>(d, s, l1, l2)];
          pp += b * snb[f][l1 + NPP * l2];
        }
      }
      const double pavg = wall ? pm : 0.5 * (pm + pp);
      const double* g = geo + (off + k) * 10;
      const double nrm = sqrt(g[3 * d] * g[3 * d] + g[3 * d + 1] * g[3 * d + 1] + g[3 * d + 2] * g[3 * d + 2]);
      const double sc = (s ? 1.0 : -1.0) * g[9] * pavg / nrm;
#pragma unroll
      for (int cc = 0; cc < 3; ++cc) {
        G[cc][k] = sc * g[3 * d + cc];  // w dA n_c {{p}}
        if (ENR) ev[cc] += ps[(off + k) * 4] * G[cc][k];
      }
    }
    __syncthreads();
    for (int it = tid; it < 3 * NPU * NPU; it += kCvThreads) {
      const int cc = it / (NPU * NPU), l = it - cc * NPU * NPU, l1 = l % NPU, l2 = l / NPU;
      double v = 0.0;
      for (int q2 = 0; q2 < Q2; ++q2) {
        const double b2 = t2 == 1 ? uy.S[q2][l2] : ux.S[q2][l2];
        for (int q1 = 0; q1 < Q1; ++q1) v += (t1 == 1 ? uy.S[q1][l1] : ux.S[q1][l1]) * b2 * G[cc][q1 + Q1 * q2];
      }
      acc[cc * NU3 + cv_layer<NPU>(d, s, l1, l2)] += v;
    }
    __syncthreads();
  }
  double* o = A.out + c.e * 3 * NU3;
  for (int it = tid; it < 3 * NU3; it += kCvThreads) o[it] = acc[it];
  if (ENR) {
    cv_block_sum<3>(ev, red, tid);
    if (tid < 3) A.out[A.ncell * 3 * NU3 + c.enr * 3 + tid] = ev[tid];
  }
}

// ---------------------------------------------------------------------------
// C: c = C u (pressure layout).
template <int NPU, int NPP, int NQ, int NQY, bool ENR>
__global__ __launch_bounds__(kCvThreads) void curved_divergence_kernel(const CvArgs A, int layer_lo, int nlayers) {
  constexpr int QY = ENR ? NQY : NQ;
  constexpr int NU3 = NPU * NPU * NPU, NU2 = NPU * NPU, NP3 = NPP * NPP * NPP, NPT = NQ * QY * NQ;
  constexpr int FMAX = NQ * (QY > NQ ? QY : NQ);
  constexpr auto& ux = ct::tab<NPU, NQ>;
  constexpr auto& uy = ct::tab<NPU, QY>;
  constexpr auto& px = ct::tab<NPP, NQ>;
  constexpr auto& py = ct::tab<NPP, QY>;
  __shared__ double su[3 * NU3];
  __shared__ double snb[6][3 * NU2];
  __shared__ double F[3][NPT];  // [a]: w|J| sum_d J^{-1}[a][d] u_d
  __shared__ double T[3][NPT];
  __shared__ double X1[3 * NPU * NPU * NQ], X2[3 * NPU * QY * NQ];
  __shared__ double G[FMAX];
  __shared__ double acc[NP3];
  __shared__ double sut[3], snut[6][3];
  __shared__ int64_t nbs[6], nbe[6];
  const int tid = threadIdx.x;
  const CvCell c = cv_cell<ENR>(A, blockIdx.x, layer_lo, nlayers);
  const int64_t n_poly = A.ncell * 3 * NU3;
  if (tid < 6) {
    int64_t ne;
    nbs[tid] = cv_neighbour(A, c, tid / 2, tid % 2, ne);
    nbe[tid] = ne;
  }
  for (int k = tid; k < 3 * NU3; k += kCvThreads) su[k] = A.in[c.e * 3 * NU3 + k];
  if (tid < 3) sut[tid] = ENR ? A.in[n_poly + c.enr * 3 + tid] : 0.0;
  __syncthreads();
  for (int k = tid; k < 6 * 3 * NU2; k += kCvThreads) {
    const int f = k / (3 * NU2), r = k - f * 3 * NU2, cc = r / NU2, l = r - cc * NU2;
    const int64_t nb = nbs[f];
    snb[f][r] = nb >= 0 ? A.in[nb * 3 * NU3 + cc * NU3 + cv_layer<NPU>(f / 2, 1 - f % 2, l % NPU, l / NPU)] : 0.0;
  }
  if (tid < 18) {
    const int f = tid / 3, cc = tid % 3;
    snut[f][cc] = (nbs[f] >= 0 && nbe[f] >= 0) ? A.in[n_poly + nbe[f] * 3 + cc] : 0.0;
  }
  const double* geo = A.geo + c.e * (int64_t)A.geo_stride * 10;
  const double* ps = ENR ? A.psi + c.enr * (int64_t)A.psi_pts * 4 : nullptr;
  cv_interp<NPU, NQ, QY, 3>(su, &T[0][0], X1, X2, tid);
  for (int q = tid; q < NPT; q += kCvThreads) {
    double u[3] = {T[0][q], T[1][q], T[2][q]};
    if (ENR)
#pragma unroll
      for (int d = 0; d < 3; ++d) u[d] += ps[q * 4] * sut[d];
    const double* g = geo + q * 10;
#pragma unroll
    for (int a = 0; a < 3; ++a) F[a][q] = g[9] * (g[3 * a] * u[0] + g[3 * a + 1] * u[1] + g[3 * a + 2] * u[2]);
  }
  __syncthreads();
  cv_project_grad<NPP, NQ, QY, 1>(&F[0][0], acc, X1, X2, tid);
  for (int B = tid; B < NP3; B += kCvThreads) acc[B] = -acc[B];
  __syncthreads();
  for (int f = 0; f < 6; ++f) {
    const int d = f / 2, s = f % 2;
    const int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
    const int Q1 = t1 == 1 ? QY : NQ, Q2 = t2 == 1 ? QY : NQ;
    const int off = psi_face_offset(NQ, QY, f);
    const int64_t nb = nbs[f], ne = nbe[f];
    // the neighbour's face (d, 1 - s) in its own point layout (an enriched neighbour across an
    // x- or z-face shares this cell's rule; across a y-face both tangential rules are nq)
    const int noff = psi_face_offset(NQ, NQY, 2 * d + 1 - s);
    for (int k = tid; k < Q1 * Q2; k += kCvThreads) {
      const int q1 = k % Q1, q2 = k / Q1;
      double um[3] = {0.0, 0.0, 0.0}, up[3] = {0.0, 0.0, 0.0};
      for (int l2 = 0; l2 < NPU; ++l2) {
        const double b2 = t2 == 1 ? uy.S[q2][l2] : ux.S[q2][l2];
        for (int l1 = 0; l1 < NPU; ++l1) {
          const double b = (t1 == 1 ? uy.S[q1][l1] : ux.S[q1][l1]) * b2;
          const int node = cv_layer<NPU>(d, s, l1, l2);
#pragma unroll
          for (int cc = 0; cc < 3; ++cc) {
            um[cc] += b * su[cc * NU3 + node];
            up[cc] += b * snb[f][cc * NU2 + l1 + NPU * l2];
          }
        }
      }
      if (ENR) {
        const double pm = ps[(off + k) * 4];
#pragma unroll
        for (int cc = 0; cc < 3; ++cc) um[cc] += pm * sut[cc];
      }
      if (nb >= 0 && ne >= 0) {
        const double pn = A.psi[(ne * (int64_t)A.psi_pts + noff + k) * 4];
#pragma unroll
        for (int cc = 0; cc < 3; ++cc) up[cc] += pn * snut[f][cc];
      }
      const double* g = geo + (off + k) * 10;
      const double nrm = sqrt(g[3 * d] * g[3 * d] + g[3 * d + 1] * g[3 * d + 1] + g[3 * d + 2] * g[3 * d + 2]);
      double un = 0.0;
#pragma unroll
      for (int cc = 0; cc < 3; ++cc) un += (nb >= 0 ? 0.5 * (um[cc] + up[cc]) : um[cc]) * g[3 * d + cc];
      G[k] = (s ? 1.0 : -1.0) * g[9] * un / nrm;  // w dA {{u}} . n
    }
    __syncthreads();
    for (int l = tid; l < NPP * NPP; l += kCvThreads) {
      const int l1 = l % NPP, l2 = l / NPP;
      double v = 0.0;
      for (int q2 = 0; q2 < Q2; ++q2) {
        const double b2 = t2 == 1 ? py.S[q2][l2] : px.S[q2][l2];
        for (int q1 = 0; q1 < Q1; ++q1) v += (t1 == 1 ? py.S[q1][l1] : px.S[q1][l1]) * b2 * G[q1 + Q1 * q2];
      }
      acc[cv_layer<NPP>(d, s, l1, l2)] += v;
    }
    __syncthreads();
  }
  for (int B = tid; B < NP3; B += kCvThreads) A.out[c.e * NP3 + B] = acc[B];
}

// ---------------------------------------------------------------------------
// Div-div penalty of the projection step (Sec. 4.2, eqs. div-div and tauD),
// cell-local: TAU computes tau_D,e = (int_e |u| / |e|) |e|^(1/3) dt/Cr (u the
// full velocity); otherwise out = D u with
//   D u (v) = tau_D,e (div u, div v)_e,  div u = sum_c sum_a J^{-1}[a][c] d_a u_c (+ grad psi . u~),
// and the test-function integrals sum_q sum_a d_a N_B(q) J^{-1}[a][c] f(q), f = w|J| tau_D div u.
template <int NPU, int NQ, int NQY, bool ENR, bool TAU>
__global__ __launch_bounds__(kCvThreads) void curved_divdiv_kernel(const CvArgs A, const double* tau_d,
                                                                   double dt_over_cr, int layer_lo, int nlayers) {
  constexpr int QY = ENR ? NQY : NQ;
  constexpr int NU3 = NPU * NPU * NPU, NPT = NQ * QY * NQ;
  __shared__ double su[3 * NU3];
  __shared__ double B9[9][NPT];  // d u_c / d xi_a at [3a + c], then F[c][a] = J^{-1}[a][c] f at [3c + a]
  __shared__ double X1[3 * NPU * NPU * NQ], X2[3 * NPU * QY * NQ];
  __shared__ double acc[TAU ? 1 : 3 * NU3];
  __shared__ double red[3 * (kCvThreads / 64)];
  __shared__ double sut[3];
  const int tid = threadIdx.x;
  const CvCell c = cv_cell<ENR>(A, blockIdx.x, layer_lo, nlayers);
  for (int k = tid; k < 3 * NU3; k += kCvThreads) su[k] = A.in[c.e * 3 * NU3 + k];
  if (tid < 3) sut[tid] = ENR ? A.in[A.ncell * 3 * NU3 + c.enr * 3 + tid] : 0.0;
  __syncthreads();
  const double* geo = A.geo + c.e * (int64_t)A.geo_stride * 10;
  const double* ps = ENR ? A.psi + c.enr * (int64_t)A.psi_pts * 4 : nullptr;
  if constexpr (TAU) {
    cv_interp<NPU, NQ, QY, 3>(su, &B9[0][0], X1, X2, tid);
    double v[2] = {0.0, 0.0};  // int |u|, |e|
    for (int q = tid; q < NPT; q += kCvThreads) {
      double u[3] = {B9[0][q], B9[1][q], B9[2][q]};
      if (ENR)
#pragma unroll
        for (int d = 0; d < 3; ++d) u[d] += ps[q * 4] * sut[d];
      const double w = geo[q * 10 + 9];
      v[0] += w * sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
      v[1] += w;
    }
    cv_block_sum<2>(v, red, tid);
    if (tid == 0) A.out[c.e] = v[0] / v[1] * cbrt(v[1]) * dt_over_cr;
  } else {
    const double td = tau_d[c.e];
    cv_interp<NPU, NQ, QY, 3, 0>(su, &B9[0][0], X1, X2, tid);
    cv_interp<NPU, NQ, QY, 3, 1>(su, &B9[3][0], X1, X2, tid);
    cv_interp<NPU, NQ, QY, 3, 2>(su, &B9[6][0], X1, X2, tid);
    double ev[3] = {0.0, 0.0, 0.0};
    for (int q = tid; q < NPT; q += kCvThreads) {
      const double* g = geo + q * 10;
      double div = 0.0;
#pragma unroll
      for (int cc = 0; cc < 3; ++cc)
#pragma unroll
        for (int a = 0; a < 3; ++a) div += g[3 * a + cc] * B9[3 * a + cc][q];
      if (ENR)
#pragma unroll
        for (int cc = 0; cc < 3; ++cc) div += ps[q * 4 + 1 + cc] * sut[cc];
      const double f = g[9] * td * div;
      // the same thread read all nine derivatives at q above
#pragma unroll
      for (int cc = 0; cc < 3; ++cc)
#pragma unroll
        for (int a = 0; a < 3; ++a) B9[3 * cc + a][q] = g[3 * a + cc] * f;
      if (ENR)
#pragma unroll
        for (int cc = 0; cc < 3; ++cc) ev[cc] += ps[q * 4 + 1 + cc] * f;
    }
    __syncthreads();
    cv_project_grad<NPU, NQ, QY, 3>(&B9[0][0], acc, X1, X2, tid);
    double* o = A.out + c.e * 3 * NU3;
    for (int it = tid; it < 3 * NU3; it += kCvThreads) o[it] = acc[it];
    if (ENR) {
      cv_block_sum<3>(ev, red, tid);
      if (tid < 3) A.out[A.ncell * 3 * NU3 + c.enr * 3 + tid] = ev[tid];
    }
  }
}

// ---------------------------------------------------------------------------
// Inverse velocity mass matrix on the curved-wall mesh, x = M^{-1} r per cell
// and component.  A curved cell's polynomial block A_BB' = sum_q W(q) N_B N_B'
// (W = w |det J|) has no tensor-product inverse, so it is solved by
// preconditioned CG, all right-hand sides of the cell at once, with the
// tensor inverse of the reference mass matrix scaled by the cell volume,
// K^{-1} / |e|, as the preconditioner (|det J| varies mildly over a cell, so
// a few tens of iterations reach the rounding floor).  An enriched cell adds
// a = A^{-1} (N, psi)_W as a fourth right-hand side and eliminates its psi
// row through the Schur complement s = (psi - sum_B a_B N_B, same)_W, formed
// pointwise as on flat cells:
//   x_psi = (r_psi - (N psi)_W . y) / s,  x_poly = y - a x_psi,  y = A^{-1} r_poly,
// x_psi = 0 while the cell's enrichment is switched off.  The cell's inputs
// are read before any output is written, so x may be r.
constexpr int kCvMaxIt = 100;
constexpr double kCvTol = 1e-15;

// Y = A P for NV vectors, A_BB' = sum_q W(q) N_B(q) N_B'(q): interpolation to the
// points and the transposed projection, each by three 1-D sweeps (x, y, z);
// X1 (NV NPU^2 NQ) and X2 (NV NPU QY NQ) are scratch.
template <int NPU, int NQ, int QY, int NV>
__device__ __forceinline__ void cv_mass_apply(const double (*P)[NPU * NPU * NPU], double (*Y)[NPU * NPU * NPU],
                                              double (*T)[NQ * QY * NQ], const double* W, double* X1, double* X2,
                                              int tid) {
  constexpr int NU3 = NPU * NPU * NPU, NPT = NQ * QY * NQ;
  constexpr int S1 = NPU * NPU * NQ, S2 = NPU * QY * NQ;
  constexpr auto& ux = ct::tab<NPU, NQ>;
  constexpr auto& uy = ct::tab<NPU, QY>;
  // x: X1[r][k][j][qx] = sum_i S[qx][i] P[r][i, j, k]
  for (int it = tid; it < NV * S1; it += kCvThreads) {
    const int r = it / S1, t = it - r * S1, qx = t % NQ, jk = t / NQ;
    double v = 0.0;
    for (int i = 0; i < NPU; ++i) v += ux.S[qx][i] * P[r][i + NPU * jk];
    X1[it] = v;
  }
  __syncthreads();
  // y: X2[r][k][qy][qx] = sum_j Sy[qy][j] X1[r][k][j][qx]
  for (int it = tid; it < NV * S2; it += kCvThreads) {
    const int r = it / S2, t = it - r * S2, qx = t % NQ, qy = (t / NQ) % QY, k = t / (NQ * QY);
    double v = 0.0;
    for (int j = 0; j < NPU; ++j) v += uy.S[qy][j] * X1[r * S1 + qx + NQ * (j + NPU * k)];
    X2[it] = v;
  }
  __syncthreads();
  // z, times W: T[r][q] = W(q) sum_k S[qz][k] X2[r][k][qy][qx]
  for (int it = tid; it < NV * NPT; it += kCvThreads) {
    const int r = it / NPT, q = it - r * NPT, qxy = q % (NQ * QY), qz = q / (NQ * QY);
    double v = 0.0;
    for (int k = 0; k < NPU; ++k) v += ux.S[qz][k] * X2[r * S2 + qxy + NQ * QY * k];
    T[r][q] = W[q] * v;
  }
  __syncthreads();
  // transposed x: X2[r][qz][qy][i] = sum_qx S[qx][i] T[r][qx, qy, qz]
  for (int it = tid; it < NV * S2; it += kCvThreads) {
    const int r = it / S2, t = it - r * S2, i = t % NPU, qyz = t / NPU;
    double v = 0.0;
    for (int qx = 0; qx < NQ; ++qx) v += ux.S[qx][i] * T[r][qx + NQ * qyz];
    X2[it] = v;
  }
  __syncthreads();
  // transposed y: X1[r][qz][j][i] = sum_qy Sy[qy][j] X2[r][qz][qy][i]
  for (int it = tid; it < NV * S1; it += kCvThreads) {
    const int r = it / S1, t = it - r * S1, i = t % NPU, j = (t / NPU) % NPU, qz = t / (NPU * NPU);
    double v = 0.0;
    for (int qy = 0; qy < QY; ++qy) v += uy.S[qy][j] * X2[r * S2 + i + NPU * (qy + QY * qz)];
    X1[it] = v;
  }
  __syncthreads();
  // transposed z: Y[r][i, j, k] = sum_qz S[qz][k] X1[r][qz][j][i]
  for (int it = tid; it < NV * NU3; it += kCvThreads) {
    const int r = it / NU3, B = it - r * NU3, ij = B % (NPU * NPU), k = B / (NPU * NPU);
    double v = 0.0;
    for (int qz = 0; qz < NQ; ++qz) v += ux.S[qz][k] * X1[r * S1 + ij + NPU * NPU * qz];
    Y[r][B] = v;
  }
  __syncthreads();
}

// z = (K^{-1} r) / vol with K^{-1} = Mi (x) Mi (x) Mi; t1, t2: scratch of NV * NU3.
template <int NPU, int NV>
__device__ __forceinline__ void cv_precond(const double (*R)[NPU * NPU * NPU], double (*Z)[NPU * NPU * NPU],
                                           double* t1, double* t2, const double* Mi, double vol, int tid) {
  constexpr int NU3 = NPU * NPU * NPU;
  for (int it = tid; it < NV * NU3; it += kCvThreads) {
    const int r = it / NU3, B = it - r * NU3, i = B % NPU, rest = B - i;
    double s = 0.0;
    for (int a = 0; a < NPU; ++a) s += Mi[i * NPU + a] * R[r][rest + a];
    t1[it] = s;
  }
  __syncthreads();
  for (int it = tid; it < NV * NU3; it += kCvThreads) {
    const int r = it / NU3, B = it - r * NU3, j = (B / NPU) % NPU, rest = B - j * NPU;
    double s = 0.0;
    for (int a = 0; a < NPU; ++a) s += Mi[j * NPU + a] * t1[r * NU3 + rest + a * NPU];
    t2[it] = s;
  }
  __syncthreads();
  for (int it = tid; it < NV * NU3; it += kCvThreads) {
    const int r = it / NU3, B = it - r * NU3, k = B / (NPU * NPU), rest = B - k * NPU * NPU;
    double s = 0.0;
    for (int a = 0; a < NPU; ++a) s += Mi[k * NPU + a] * t2[r * NU3 + rest + a * NPU * NPU];
    Z[r][B] = s / vol;
  }
  __syncthreads();
}

template <int NPU, int NQ, int NQY, bool ENR>
__global__ __launch_bounds__(kCvThreads) void curved_invmass_kernel(const CvArgs A, const double* minv,
                                                                    const int32_t* act, int layer_lo, int nlayers) {
  constexpr int QY = ENR ? NQY : NQ;
  constexpr int NU3 = NPU * NPU * NPU, NPT = NQ * QY * NQ, NV = ENR ? 4 : 3;
  constexpr auto& ux = ct::tab<NPU, NQ>;
  constexpr auto& uy = ct::tab<NPU, QY>;
  __shared__ double X[NV][NU3], R[NV][NU3], Z[NV][NU3], P[NV][NU3], AP[NV][NU3];
  __shared__ double T[NV][NPT];
  __shared__ double W[NPT], PS[ENR ? NPT : 1], B0[ENR ? NU3 : 1];
  __shared__ double Mi[NPU * NPU];
  __shared__ double X1[NV * NPU * NPU * NQ], X2[NV * NPU * QY * NQ];
  __shared__ double red[3 * NV * (kCvThreads / 64)];
  __shared__ double rhs_e[3];
  const int tid = threadIdx.x;
  const CvCell c = cv_cell<ENR>(A, blockIdx.x, layer_lo, nlayers);
  const double* geo = A.geo + c.e * (int64_t)A.geo_stride * 10;
  const double* ps = ENR ? A.psi + c.enr * (int64_t)A.psi_pts * 4 : nullptr;
  const int64_t n_poly = A.ncell * 3 * NU3;
  for (int k = tid; k < NPU * NPU; k += kCvThreads) Mi[k] = minv[k];
  for (int k = tid; k < 3 * NU3; k += kCvThreads) R[k / NU3][k % NU3] = A.in[c.e * 3 * NU3 + k];
  if (ENR && tid < 3) rhs_e[tid] = A.in[n_poly + c.enr * 3 + tid];
  double vv[1] = {0.0};
  for (int q = tid; q < NPT; q += kCvThreads) {
    W[q] = geo[q * 10 + 9];
    vv[0] += W[q];
    if (ENR) {
      PS[q] = ps[q * 4];
      T[0][q] = W[q] * PS[q];
    }
  }
  cv_block_sum<1>(vv, red, tid);  // (ends with the barrier the loads need)
  const double vol = vv[0];
  if (ENR) {
    // fourth right-hand side (N_B, psi)_W
    for (int B = tid; B < NU3; B += kCvThreads) {
      const int i = B % NPU, j = (B / NPU) % NPU, k = B / (NPU * NPU);
      double s = 0.0;
      for (int qz = 0; qz < NQ; ++qz)
        for (int qy = 0; qy < QY; ++qy) {
          const double yz = uy.S[qy][j] * ux.S[qz][k];
          for (int qx = 0; qx < NQ; ++qx) s += ux.S[qx][i] * yz * T[0][qx + NQ * (qy + QY * qz)];
        }
      R[3][B] = s;
      B0[B] = s;
    }
    __syncthreads();
  }
  // PCG from x = 0 on all NV right-hand sides
  for (int k = tid; k < NV * NU3; k += kCvThreads) X[k / NU3][k % NU3] = 0.0;
  cv_precond<NPU, NV>(R, Z, &T[0][0], &AP[0][0], Mi, vol, tid);
  double rz[NV], bb[NV];
  {
    double v[2 * NV] = {};
    for (int k = tid; k < NV * NU3; k += kCvThreads) {
      const int r = k / NU3, B = k - r * NU3;
      v[r] += R[r][B] * Z[r][B];
      v[NV + r] += R[r][B] * R[r][B];
      P[r][B] = Z[r][B];
    }
    cv_block_sum<2 * NV>(v, red, tid);
#pragma unroll
    for (int r = 0; r < NV; ++r) {
      rz[r] = v[r];
      bb[r] = v[NV + r];
    }
  }
  bool done[NV];
#pragma unroll
  for (int r = 0; r < NV; ++r) done[r] = !(bb[r] > 0.0);
  for (int it = 0; it < kCvMaxIt; ++it) {
    bool all = true;
#pragma unroll
    for (int r = 0; r < NV; ++r) all = all && done[r];
    if (all) break;
    cv_mass_apply<NPU, NQ, QY, NV>(P, AP, T, W, X1, X2, tid);
    double pa[NV] = {};
    for (int k = tid; k < NV * NU3; k += kCvThreads) {
      const int r = k / NU3, B = k - r * NU3;
      pa[r] += P[r][B] * AP[r][B];
    }
    cv_block_sum<NV>(pa, red, tid);
    double al[NV];
#pragma unroll
    for (int r = 0; r < NV; ++r) al[r] = (done[r] || !(pa[r] > 0.0)) ? 0.0 : rz[r] / pa[r];
    for (int k = tid; k < NV * NU3; k += kCvThreads) {
      const int r = k / NU3, B = k - r * NU3;
      X[r][B] += al[r] * P[r][B];
      R[r][B] -= al[r] * AP[r][B];
    }
    __syncthreads();
    cv_precond<NPU, NV>(R, Z, &T[0][0], &AP[0][0], Mi, vol, tid);
    double v[2 * NV] = {};
    for (int k = tid; k < NV * NU3; k += kCvThreads) {
      const int r = k / NU3, B = k - r * NU3;
      v[r] += R[r][B] * Z[r][B];
      v[NV + r] += R[r][B] * R[r][B];
    }
    cv_block_sum<2 * NV>(v, red, tid);
    double be[NV];
#pragma unroll
    for (int r = 0; r < NV; ++r) {
      if (!done[r] && (al[r] == 0.0 || v[NV + r] <= kCvTol * kCvTol * bb[r])) done[r] = true;
      be[r] = (done[r] || !(rz[r] > 0.0)) ? 0.0 : v[r] / rz[r];
      if (!done[r]) rz[r] = v[r];
    }
    for (int k = tid; k < NV * NU3; k += kCvThreads) {
      const int r = k / NU3, B = k - r * NU3;
      if (!done[r]) P[r][B] = Z[r][B] + be[r] * P[r][B];
    }
    __syncthreads();
  }
  double* o = A.out + c.e * 3 * NU3;
  if (ENR) {
    // r_psi = psi - sum_B a_B N_B at the points; s = (r_psi, r_psi)_W; b . y_c
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    for (int q = tid; q < NPT; q += kCvThreads) {
      const int qx = q % NQ, qy = (q / NQ) % QY, qz = q / (NQ * QY);
      double pa = 0.0;
      for (int k = 0; k < NPU; ++k)
        for (int j = 0; j < NPU; ++j) {
          const double fy = uy.S[qy][j] * ux.S[qz][k];
          for (int i = 0; i < NPU; ++i) pa += ux.S[qx][i] * fy * X[3][i + NPU * (j + NPU * k)];
        }
      const double rp = PS[q] - pa;
      v[0] += W[q] * rp * rp;
    }
    for (int B = tid; B < NU3; B += kCvThreads)
#pragma unroll
      for (int cc = 0; cc < 3; ++cc) v[1 + cc] += B0[B] * X[cc][B];
    cv_block_sum<4>(v, red, tid);
    const bool on = act[c.enr] != 0 && v[0] > 0.0;
    double xe[3];
#pragma unroll
    for (int cc = 0; cc < 3; ++cc) xe[cc] = on ? (rhs_e[cc] - v[1 + cc]) / v[0] : 0.0;
    for (int k = tid; k < 3 * NU3; k += kCvThreads) {
      const int cc = k / NU3, B = k - cc * NU3;
      o[k] = X[cc][B] - X[3][B] * xe[cc];
    }
    if (tid < 3) A.out[n_poly + c.enr * 3 + tid] = xe[tid];
  } else {
    for (int k = tid; k < 3 * NU3; k += kCvThreads) o[k] = X[k / NU3][k % NU3];
  }
}

// ---------------------------------------------------------------------------
// Right-hand side of the projected vorticity (Sec. 4.2), b(v) = (v, curl u)_e
// for v = N_B e_c and, in enriched cells, psi e_c; grad u = J^{-T} grad_xi u
// point by point (plus u~ (x) grad psi in enriched cells).
template <int NPU, int NQ, int NQY, bool ENR>
__global__ __launch_bounds__(kCvThreads) void curved_vort_rhs_kernel(const CvArgs A, int layer_lo, int nlayers) {
  constexpr int QY = ENR ? NQY : NQ;
  constexpr int NU3 = NPU * NPU * NPU, NPT = NQ * QY * NQ;
  __shared__ double su[3 * NU3];
  __shared__ double B9[9][NPT];  // d u_c / d xi_a at [3a + c]; then w|J| (curl u)_c at [c]
  __shared__ double X1[3 * NPU * NPU * NQ], X2[3 * NPU * QY * NQ];
  __shared__ double acc[3 * NU3];
  __shared__ double red[3 * (kCvThreads / 64)];
  __shared__ double sut[3];
  const int tid = threadIdx.x;
  const CvCell c = cv_cell<ENR>(A, blockIdx.x, layer_lo, nlayers);
  for (int k = tid; k < 3 * NU3; k += kCvThreads) su[k] = A.in[c.e * 3 * NU3 + k];
  if (tid < 3) sut[tid] = ENR ? A.in[A.ncell * 3 * NU3 + c.enr * 3 + tid] : 0.0;
  __syncthreads();
  const double* geo = A.geo + c.e * (int64_t)A.geo_stride * 10;
  const double* ps = ENR ? A.psi + c.enr * (int64_t)A.psi_pts * 4 : nullptr;
  cv_interp<NPU, NQ, QY, 3, 0>(su, &B9[0][0], X1, X2, tid);
  cv_interp<NPU, NQ, QY, 3, 1>(su, &B9[3][0], X1, X2, tid);
  cv_interp<NPU, NQ, QY, 3, 2>(su, &B9[6][0], X1, X2, tid);
  double ev[3] = {0.0, 0.0, 0.0};
  for (int q = tid; q < NPT; q += kCvThreads) {
    const double* g = geo + q * 10;
    double gr[3][3];  // [c][d] = d u_c / d x_d
#pragma unroll
    for (int cc = 0; cc < 3; ++cc)
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        gr[cc][d] = g[d] * B9[cc][q] + g[3 + d] * B9[3 + cc][q] + g[6 + d] * B9[6 + cc][q];
        if (ENR) gr[cc][d] += sut[cc] * ps[q * 4 + 1 + d];
      }
    const double w = g[9];
    const double cu[3] = {w * (gr[2][1] - gr[1][2]), w * (gr[0][2] - gr[2][0]), w * (gr[1][0] - gr[0][1])};
    // the same thread read all nine derivatives at q above
#pragma unroll
    for (int cc = 0; cc < 3; ++cc) {
      B9[cc][q] = cu[cc];
      if (ENR) ev[cc] += ps[q * 4] * cu[cc];
    }
  }
  __syncthreads();
  cv_project_vals<NPU, NQ, QY, 3>(&B9[0][0], acc, X1, X2, tid);
  double* o = A.out + c.e * 3 * NU3;
  for (int it = tid; it < 3 * NU3; it += kCvThreads) o[it] = acc[it];
  if (ENR) {
    cv_block_sum<3>(ev, red, tid);
    if (tid < 3) A.out[A.ncell * 3 * NU3 + c.enr * 3 + tid] = ev[tid];
  }
}

// ---------------------------------------------------------------------------
// Wall term of the pressure equation with the high-order Neumann data
// (Sec. 4.1, eq. bc_d_pres) on the curved-wall mesh, ADDED into rhs:
//   rhs(q) += int_wall q h_N dA,  h_N = -(sum_h beta_h (div(u_h (x) u_h) + nu curl omega_h) - f) . n,
// div(u (x) u) = (u . grad) u + u div u, n dA = +-|det J| J^{-T} e_y dA_ref on the
// wall faces (all three components: the lower wall is curved).  One workgroup
// per wall cell, one thread per face point; each cell adds only into its own
// wall-face layer.
struct CvNeuArgs {
  const double* u[2];
  const double* om[2];
  double beta[2], f[3], nu;
  int nh;
};

template <int NPU, int NPP, int NQ, int NQY>
__global__ __launch_bounds__(64) void curved_neumann_kernel(const CvArgs A, const CvNeuArgs N, double* rhs) {
  constexpr int NU3 = NPU * NPU * NPU, NP3 = NPP * NPP * NPP, NF = NQ * NQ;
  constexpr auto& ux = ct::tab<NPU, NQ>;
  constexpr auto& px = ct::tab<NPP, NQ>;
  __shared__ double su[2][2][3 * NU3];  // [history][u, omega]
  __shared__ double st[2][2][3];
  __shared__ double H[NF];
  const int tid = threadIdx.x;
  const int b = blockIdx.x, wall = b / (A.nx * A.nz), col = b - wall * A.nx * A.nz;
  const int ex = col % A.nx, ez = col / A.nx, ey = wall ? A.ny - 1 : 0, s = wall;
  const int64_t e = ex + (int64_t)A.nx * (ey + (int64_t)A.ny * ez);
  const int64_t enr = cv_enr(A, ex, ey, ez);
  const int64_t n_poly = A.ncell * 3 * NU3;
  for (int h = 0; h < N.nh; ++h)
    for (int k = tid; k < 3 * NU3; k += 64) {
      su[h][0][k] = N.u[h][e * 3 * NU3 + k];
      su[h][1][k] = N.om[h][e * 3 * NU3 + k];
    }
  if (tid < 6 * N.nh) {
    const int h = tid / 6, w = (tid / 3) % 2, cc = tid % 3;
    st[h][w][cc] = enr >= 0 ? (w ? N.om[h] : N.u[h])[n_poly + enr * 3 + cc] : 0.0;
  }
  __syncthreads();
  const int qyc = enr >= 0 ? NQY : NQ;
  const double* g = A.geo + (e * A.geo_stride + psi_face_offset(NQ, qyc, 2 + s)) * 10;
  const double* ps = enr >= 0 ? A.psi + (enr * A.psi_pts + psi_face_offset(NQ, NQY, 2 + s)) * 4 : nullptr;
  const double* nd = s ? ux.nd1 : ux.nd0;
  const int jf = s ? NPU - 1 : 0;
  for (int q = tid; q < NF; q += 64) {
    const int qx = q % NQ, qz = q / NQ;
    const double* gq = g + q * 10;
    double hv[3] = {0.0, 0.0, 0.0};
    for (int h = 0; h < N.nh; ++h) {
      double val[3] = {}, du[2][3][3] = {};  // [u, omega][c][a]
      for (int k = 0; k < NPU; ++k)
        for (int i = 0; i < NPU; ++i) {
          const double bxz = ux.S[qx][i] * ux.S[qz][k], dx = ux.Sd[qx][i] * ux.S[qz][k];
          const double dz = ux.S[qx][i] * ux.Sd[qz][k];
          for (int w = 0; w < 2; ++w)
#pragma unroll
            for (int cc = 0; cc < 3; ++cc) {
              const double v = su[h][w][cc * NU3 + i + NPU * (jf + NPU * k)];
              if (w == 0) val[cc] += bxz * v;
              du[w][cc][0] += dx * v;
              du[w][cc][2] += dz * v;
              double dy = 0.0;
              for (int j = 0; j < NPU; ++j) dy += nd[j] * su[h][w][cc * NU3 + i + NPU * (j + NPU * k)];
              du[w][cc][1] += bxz * dy;
            }
        }
      double gr[2][3][3];
      for (int w = 0; w < 2; ++w)
#pragma unroll
        for (int cc = 0; cc < 3; ++cc)
#pragma unroll
          for (int d = 0; d < 3; ++d) {
            gr[w][cc][d] = gq[d] * du[w][cc][0] + gq[3 + d] * du[w][cc][1] + gq[6 + d] * du[w][cc][2];
            if (ps) gr[w][cc][d] += st[h][w][cc] * ps[q * 4 + 1 + d];
          }
      if (ps)
#pragma unroll
        for (int cc = 0; cc < 3; ++cc) val[cc] += ps[q * 4] * st[h][0][cc];
      const double div = gr[0][0][0] + gr[0][1][1] + gr[0][2][2];
      const double curl[3] = {gr[1][2][1] - gr[1][1][2], gr[1][0][2] - gr[1][2][0], gr[1][1][0] - gr[1][0][1]};
#pragma unroll
      for (int cc = 0; cc < 3; ++cc)
        hv[cc] += N.beta[h] * (gr[0][cc][0] * val[0] + gr[0][cc][1] * val[1] + gr[0][cc][2] * val[2] +
                               val[cc] * div + N.nu * curl[cc]);
    }
    // n w dA = +-(w dA) J^{-T} e_y / |J^{-T} e_y|
    const double nrm = sqrt(gq[3] * gq[3] + gq[4] * gq[4] + gq[5] * gq[5]);
    const double sc = (s ? 1.0 : -1.0) * gq[9] / nrm;
    H[q] = -sc * ((hv[0] - N.f[0]) * gq[3] + (hv[1] - N.f[1]) * gq[4] + (hv[2] - N.f[2]) * gq[5]);
  }
  __syncthreads();
  for (int l = tid; l < NPP * NPP; l += 64) {
    const int i = l % NPP, k = l / NPP;
    double v = 0.0;
    for (int qz = 0; qz < NQ; ++qz)
      for (int qx = 0; qx < NQ; ++qx) v += px.S[qx][i] * px.S[qz][k] * H[qx + NQ * qz];
    rhs[e * NP3 + cv_layer<NPP>(1, s, i, k)] += v;
  }
}

}  // namespace

// (k_u+1, nq_u, nq_wn) combinations of the velocity operators
#define DG_CVD_COMBOS(X) X(3, 4, 8) X(3, 4, 4) X(4, 4, 8) X(4, 5, 8) X(4, 5, 5) X(5, 7, 8) X(6, 8, 8)

int launch_vorticity_rhs_curved(const dg_mesh* m, const double* u, double* b, hipStream_t s) {
  CvArgs A;
  A.nx = m->P.nx;
  A.ny = m->P.ny;
  A.nz = m->P.nz;
  A.lower_slot = m->lower_slot;
  A.upper_slot = m->upper_slot;
  A.nslots = m->n_enr_layers;
  A.psi_pts = m->psi_pts;
  A.geo_stride = m->geo_stride;
  A.fully_periodic = m->P.fully_periodic;
  A.ncell = m->ncell;
  A.geo = m->geo;
  A.psi = m->psi;
  A.in = u;
  A.out = b;
  if (!m->geo || m->nle != 1) return set_error(DG_ERR_UNSUPPORTED, "curved vorticity: l = 0 enrichment only");
  const int lo = (m->P.fully_periodic || m->lower_slot < 0) ? 0 : 1;
  const int hi = (m->P.fully_periodic || m->upper_slot < 0) ? m->P.ny - 1 : m->P.ny - 2;
  const int nl = hi - lo + 1;
  const int64_t nreg = nl > 0 ? (int64_t)m->P.nx * nl * m->P.nz : 0;
  const bool any_w = m->nenr == 0;
  const int nqw = m->P.nq_wn;
#define X(p, q, w)                                                                                          \
  if (m->np_u == p && m->P.nq_u == q && (any_w || nqw == w)) {                                              \
    if (nreg > 0) {                                                                                         \
      hipLaunchKernelGGL((curved_vort_rhs_kernel<p, q, w, false>), dim3((unsigned)nreg), dim3(kCvThreads), 0, s, \
                         A, lo, nl);                                                                        \
      const int rc = check_hip(hipGetLastError(), "curved vorticity kernel launch");                        \
      if (rc) return rc;                                                                                    \
    }                                                                                                       \
    if (m->nenr > 0)                                                                                        \
      hipLaunchKernelGGL((curved_vort_rhs_kernel<p, q, w, true>), dim3((unsigned)m->nenr), dim3(kCvThreads), 0, \
                         s, A, 0, 0);                                                                       \
    return check_hip(hipGetLastError(), "curved vorticity kernel launch");                                  \
  }
  DG_CVD_COMBOS(X)
#undef X
  return set_error(DG_ERR_UNSUPPORTED, "curved vorticity: (k_u+1, nq_u, nq_wn) combination not compiled");
}

int launch_inverse_mass_curved(const dg_mesh* m, const double* r, double* x, hipStream_t s) {
  CvArgs A;
  A.nx = m->P.nx;
  A.ny = m->P.ny;
  A.nz = m->P.nz;
  A.lower_slot = m->lower_slot;
  A.upper_slot = m->upper_slot;
  A.nslots = m->n_enr_layers;
  A.psi_pts = m->psi_pts;
  A.geo_stride = m->geo_stride;
  A.fully_periodic = m->P.fully_periodic;
  A.ncell = m->ncell;
  A.geo = m->geo;
  A.psi = m->psi;
  A.in = r;
  A.out = x;
  if (!m->geo || m->nle != 1) return set_error(DG_ERR_UNSUPPORTED, "curved inverse mass: l = 0 enrichment only");
  const int lo = (m->P.fully_periodic || m->lower_slot < 0) ? 0 : 1;
  const int hi = (m->P.fully_periodic || m->upper_slot < 0) ? m->P.ny - 1 : m->P.ny - 2;
  const int nl = hi - lo + 1;
  const int64_t nreg = nl > 0 ? (int64_t)m->P.nx * nl * m->P.nz : 0;
  const bool any_w = m->nenr == 0;
  const int nqw = m->P.nq_wn;
#define X(p, q, w)                                                                                          \
  if (m->np_u == p && m->P.nq_u == q && (any_w || nqw == w)) {                                              \
    if (nreg > 0) {                                                                                         \
      hipLaunchKernelGGL((curved_invmass_kernel<p, q, w, false>), dim3((unsigned)nreg), dim3(kCvThreads), 0, s, \
                         A, m->minv, m->act, lo, nl);                                                       \
      const int rc = check_hip(hipGetLastError(), "curved inverse mass kernel launch");                     \
      if (rc) return rc;                                                                                    \
    }                                                                                                       \
    if (m->nenr > 0)                                                                                        \
      hipLaunchKernelGGL((curved_invmass_kernel<p, q, w, true>), dim3((unsigned)m->nenr), dim3(kCvThreads), 0, \
                         s, A, m->minv, m->act, 0, 0);                                                      \
    return check_hip(hipGetLastError(), "curved inverse mass kernel launch");                               \
  }
  DG_CVD_COMBOS(X)
#undef X
  return set_error(DG_ERR_UNSUPPORTED, "curved inverse mass: (k_u+1, nq_u, nq_wn) combination not compiled");
}


int launch_divdiv_curved(const dg_mesh* m, bool tau, const double* u, const double* tau_d, double dt_over_cr,
                         double* out, hipStream_t s) {
  CvArgs A;
  A.nx = m->P.nx;
  A.ny = m->P.ny;
  A.nz = m->P.nz;
  A.lower_slot = m->lower_slot;
  A.upper_slot = m->upper_slot;
  A.nslots = m->n_enr_layers;
  A.psi_pts = m->psi_pts;
  A.geo_stride = m->geo_stride;
  A.fully_periodic = m->P.fully_periodic;
  A.ncell = m->ncell;
  A.geo = m->geo;
  A.psi = m->psi;
  A.in = u;
  A.out = out;
  if (!m->geo || m->nle != 1) return set_error(DG_ERR_UNSUPPORTED, "curved div-div: l = 0 enrichment only");
  const int lo = (m->P.fully_periodic || m->lower_slot < 0) ? 0 : 1;
  const int hi = (m->P.fully_periodic || m->upper_slot < 0) ? m->P.ny - 1 : m->P.ny - 2;
  const int nl = hi - lo + 1;
  const int64_t nreg = nl > 0 ? (int64_t)m->P.nx * nl * m->P.nz : 0;
  const bool any_w = m->nenr == 0;
  const int nqw = m->P.nq_wn;
#define LAUNCH(p, q, w, ENRV, TAUV, grid, lo_, nl_)                                                       \
  hipLaunchKernelGGL((curved_divdiv_kernel<p, q, w, ENRV, TAUV>), dim3((unsigned)(grid)), dim3(kCvThreads), 0, s, \
                     A, tau_d, dt_over_cr, lo_, nl_)
#define X(p, q, w)                                                                                      \
  if (m->np_u == p && m->P.nq_u == q && (any_w || nqw == w)) {                                          \
    if (nreg > 0) {                                                                                     \
      if (tau) LAUNCH(p, q, w, false, true, nreg, lo, nl);                                              \
      else LAUNCH(p, q, w, false, false, nreg, lo, nl);                                                 \
      const int rc = check_hip(hipGetLastError(), "curved div-div kernel launch");                      \
      if (rc) return rc;                                                                                \
    }                                                                                                   \
    if (m->nenr > 0) {                                                                                  \
      if (tau) LAUNCH(p, q, w, true, true, m->nenr, 0, 0);                                              \
      else LAUNCH(p, q, w, true, false, m->nenr, 0, 0);                                                 \
    }                                                                                                   \
    return check_hip(hipGetLastError(), "curved div-div kernel launch");                                \
  }
  DG_CVD_COMBOS(X)
#undef X
#undef LAUNCH
  return set_error(DG_ERR_UNSUPPORTED, "curved div-div penalty: (k_u+1, nq_u, nq_wn) combination not compiled");
}

// (k_u+1, k_p+1, nq_u, nq_wn) combinations: the velocity ones with k_p = k_u - 1
#define DG_CV_COMBOS(X) X(3, 2, 4, 8) X(3, 2, 4, 4) X(4, 3, 4, 8) X(4, 3, 5, 8) X(4, 3, 5, 5) X(5, 4, 7, 8) X(6, 5, 8, 8)

int launch_pressure_neumann_curved(const dg_mesh* m, int nh, const double* const* us, const double* const* oms,
                                   const double* beta, const double* f, double* rhs, hipStream_t s) {
  CvArgs A;
  A.nx = m->P.nx;
  A.ny = m->P.ny;
  A.nz = m->P.nz;
  A.lower_slot = m->lower_slot;
  A.upper_slot = m->upper_slot;
  A.nslots = m->n_enr_layers;
  A.psi_pts = m->psi_pts;
  A.geo_stride = m->geo_stride;
  A.fully_periodic = m->P.fully_periodic;
  A.ncell = m->ncell;
  A.geo = m->geo;
  A.psi = m->psi;
  A.in = nullptr;
  A.out = nullptr;
  if (!m->geo || m->nle != 1) return set_error(DG_ERR_UNSUPPORTED, "curved Neumann data: l = 0 enrichment only");
  CvNeuArgs N{};
  for (int h = 0; h < nh; ++h) {
    N.u[h] = us[h];
    N.om[h] = oms[h];
    N.beta[h] = beta[h];
  }
  N.nh = nh;
  for (int d = 0; d < 3; ++d) N.f[d] = f ? f[d] : 0.0;
  N.nu = m->P.nu;
  const unsigned g = (unsigned)(2 * m->P.nx * m->P.nz);
  const bool any_w = m->nenr == 0;
  const int nqw = m->P.nq_wn;
#define X(pu, pp, q, w)                                                                                  \
  if (m->np_u == pu && m->np_p == pp && m->P.nq_u == q && (any_w || nqw == w)) {                          \
    hipLaunchKernelGGL((curved_neumann_kernel<pu, pp, q, w>), dim3(g), dim3(64), 0, s, A, N, rhs);       \
    return check_hip(hipGetLastError(), "curved pressure Neumann launch");                               \
  }
  DG_CV_COMBOS(X)
#undef X
  return set_error(DG_ERR_UNSUPPORTED, "curved Neumann data: (k_u+1, k_p+1, nq_u, nq_wn) combination not compiled");
}

int launch_divgrad_curved(const dg_mesh* m, bool divergence, const double* in, double* out, hipStream_t s) {
  CvArgs A;
  A.nx = m->P.nx;
  A.ny = m->P.ny;
  A.nz = m->P.nz;
  A.lower_slot = m->lower_slot;
  A.upper_slot = m->upper_slot;
  A.nslots = m->n_enr_layers;
  A.psi_pts = m->psi_pts;
  A.geo_stride = m->geo_stride;
  A.fully_periodic = m->P.fully_periodic;
  A.ncell = m->ncell;
  A.geo = m->geo;
  A.psi = m->psi;
  A.in = in;
  A.out = out;
  if (!m->geo || m->nle != 1) return set_error(DG_ERR_UNSUPPORTED, "curved P / C: l = 0 enrichment only");
  const int lo = (m->P.fully_periodic || m->lower_slot < 0) ? 0 : 1;
  const int hi = (m->P.fully_periodic || m->upper_slot < 0) ? m->P.ny - 1 : m->P.ny - 2;
  const int nl = hi - lo + 1;
  const int64_t nreg = nl > 0 ? (int64_t)m->P.nx * nl * m->P.nz : 0;
  const bool any_w = m->nenr == 0;
  const int nqw = m->P.nq_wn;
#define LAUNCH(KER, pu, pp, q, w, ENRV, grid, lo_, nl_) \
  hipLaunchKernelGGL((KER<pu, pp, q, w, ENRV>), dim3((unsigned)(grid)), dim3(kCvThreads), 0, s, A, lo_, nl_)
#define X(pu, pp, q, w)                                                                               \
  if (m->np_u == pu && m->np_p == pp && m->P.nq_u == q && (any_w || nqw == w)) {                      \
    if (nreg > 0) {                                                                                   \
      if (divergence) LAUNCH(curved_divergence_kernel, pu, pp, q, w, false, nreg, lo, nl);            \
      else LAUNCH(curved_gradient_kernel, pu, pp, q, w, false, nreg, lo, nl);                         \
      const int rc = check_hip(hipGetLastError(), "curved divergence/gradient kernel launch");        \
      if (rc) return rc;                                                                              \
    }                                                                                                 \
    if (m->nenr > 0) {                                                                                \
      if (divergence) LAUNCH(curved_divergence_kernel, pu, pp, q, w, true, m->nenr, 0, 0);            \
      else LAUNCH(curved_gradient_kernel, pu, pp, q, w, true, m->nenr, 0, 0);                         \
    }                                                                                                 \
    return check_hip(hipGetLastError(), "curved divergence/gradient kernel launch");                  \
  }
  DG_CV_COMBOS(X)
#undef X
#undef LAUNCH
  return set_error(DG_ERR_UNSUPPORTED,
                   "curved pressure gradient / velocity divergence: (k_u+1, k_p+1, nq_u, nq_wn) combination not compiled");
}

}  // namespace dgwm
