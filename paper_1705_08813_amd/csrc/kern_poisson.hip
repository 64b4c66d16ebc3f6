// SIP Poisson operator (arXiv 1705.08813, Sec. 4.2, pressure Laplace term
// with flux eq. ipflux and homogeneous Neumann walls), matrix-free:
//   (A p)(q) = sum_e (grad q, grad p)_e
//            + sum_F [ -1/2 (grad q.n)(p- - p+) - q ({{grad p}}.n - tau_F (p- - p+)) ]_F
// and the Jacobi diagonal of A.  Box (affine) meshes.
//
// One workgroup per cell, sum-factorized volume term, element-by-element
// face terms (each cell reads its neighbour's nodal values), single writer
// per output entry.
#include "kern_common.h"

namespace dgwm {

namespace {

template <typename T, int NP, int NQ>
struct PoiShape {
  static constexpr int NP2 = NP * NP, NP3 = NP * NP * NP, NPTS = NQ * NQ * NQ, FP = NQ * NQ;
  static constexpr int FACE = 2 * 2 * NP2 + 2 * 2 * FP + 2 * FP;  // layers, traces, fluxes
  static constexpr int VOL = 4 * NPTS;
  static constexpr int BIG = VOL > FACE ? VOL : FACE;
};

template <typename T, int NP, int NQ, int D, int S>
__device__ __forceinline__ void poi_face(const MeshDev& M, const T* __restrict__ p, const T* s_p, T* s_r, T* s_big,
                                         int ex, int ey, int ez, T hx, T hy, T hz) {
  using Sh = PoiShape<T, NP, NQ>;
  constexpr TabLayout L = tab_layout(NP, NQ, NQ);
  constexpr int T1 = D == 0 ? 1 : 0;
  constexpr int T2 = D == 2 ? 1 : 2;
  constexpr int NP2 = Sh::NP2, NP3 = Sh::NP3, FP = Sh::FP;
  const int tid = threadIdx.x, nt = blockDim.x;
  int nidx[3] = {ex, ey, ez};
  const int nmax[3] = {M.nx, M.ny, M.nz};
  nidx[D] += S ? 1 : -1;
  if (nidx[D] < 0 || nidx[D] >= nmax[D]) {
    if (D == 1 && !M.fully_periodic) return;  // wall: homogeneous Neumann, no terms
    nidx[D] = (nidx[D] + nmax[D]) % nmax[D];
  }
  const int64_t enb = nidx[0] + (int64_t)M.nx * (nidx[1] + (int64_t)M.ny * nidx[2]);
  const double* tab = M.tab;
  const double* Sq = tab + L.S;
  const double* wq = tab + L.w;
  const double* ndo = tab + (S ? L.nd1 : L.nd0);
  const double* ndn = tab + (S ? L.nd0 : L.nd1);
  const T hown[3] = {hx, hy, hz};
  const T hd = hown[D];
  const T hdn = (D == 1) ? T(M.hy[nidx[1]]) : hd;
  const T ht1 = hown[T1], ht2 = hown[T2];
  const T tauF = T(M.pen) * (T(1) / hd > T(1) / hdn ? T(1) / hd : T(1) / hdn);
  const T sg = S ? T(1) : T(-1);

  T* lay = s_big;                  // [side][val|dn][NP2]
  T* tr = lay + 2 * 2 * NP2;       // [side][val|dn][FP]
  T* fl = tr + 2 * 2 * FP;         // [fv | fn][FP]

  for (int t = tid; t < 2 * NP2; t += nt) {
    const int side = t / NP2, k = t - side * NP2;
    const int i1 = k % NP, i2 = k / NP;
    int pos[3];
    pos[T1] = i1;
    pos[T2] = i2;
    const int lface = (side == 0 ? S : 1 - S) ? NP - 1 : 0;
    const double* nd = side == 0 ? ndo : ndn;
    T val = 0, der = 0;
#pragma unroll
    for (int l = 0; l < NP; ++l) {
      pos[D] = l;
      const int B = pos[0] + NP * (pos[1] + NP * pos[2]);
      const T x = side == 0 ? s_p[B] : p[enb * NP3 + B];
      der += T(nd[l]) * x;
      if (l == lface) val = x;
    }
    lay[(side * 2 + 0) * NP2 + k] = val;
    lay[(side * 2 + 1) * NP2 + k] = der / (side == 0 ? hd : hdn);
  }
  __syncthreads();
  for (int t = tid; t < 2 * FP; t += nt) {
    const int side = t / FP, pt = t - side * FP;
    const int q1 = pt % NQ, q2 = pt / NQ;
    const T* lv = lay + (side * 2 + 0) * NP2;
    const T* ln = lay + (side * 2 + 1) * NP2;
    T v = 0, dn = 0;
#pragma unroll
    for (int i2 = 0; i2 < NP; ++i2) {
      T av = 0, an = 0;
#pragma unroll
      for (int i1 = 0; i1 < NP; ++i1) {
        av += T(Sq[q1 * NP + i1]) * lv[i1 + NP * i2];
        an += T(Sq[q1 * NP + i1]) * ln[i1 + NP * i2];
      }
      v += T(Sq[q2 * NP + i2]) * av;
      dn += T(Sq[q2 * NP + i2]) * an;
    }
    tr[(side * 2 + 0) * FP + pt] = v;
    tr[(side * 2 + 1) * FP + pt] = dn;
  }
  __syncthreads();
  for (int pt = tid; pt < FP; pt += nt) {
    const int q1 = pt % NQ, q2 = pt / NQ;
    const T wf = T(wq[q1]) * T(wq[q2]) * ht1 * ht2;
    const T jmp = tr[0 * FP + pt] - tr[2 * FP + pt];
    const T avg_n = T(0.5) * (tr[1 * FP + pt] + tr[3 * FP + pt]) * sg;
    fl[pt] = wf * (-avg_n + tauF * jmp);     // tested with q
    fl[FP + pt] = wf * (T(-0.5) * jmp * sg); // tested with d q / d x_D
  }
  __syncthreads();
  for (int k = tid; k < NP2; k += nt) {
    const int i1 = k % NP, i2 = k / NP;
    T rv = 0, bn = 0;
#pragma unroll
    for (int q2 = 0; q2 < NQ; ++q2) {
      T a0 = 0, a1 = 0;
#pragma unroll
      for (int q1 = 0; q1 < NQ; ++q1) {
        const T s1 = T(Sq[q1 * NP + i1]);
        a0 += s1 * fl[q1 + NQ * q2];
        a1 += s1 * fl[FP + q1 + NQ * q2];
      }
      rv += T(Sq[q2 * NP + i2]) * a0;
      bn += T(Sq[q2 * NP + i2]) * a1;
    }
    int pos[3];
    pos[T1] = i1;
    pos[T2] = i2;
    const int lface = S ? NP - 1 : 0;
#pragma unroll
    for (int l = 0; l < NP; ++l) {
      pos[D] = l;
      const int B = pos[0] + NP * (pos[1] + NP * pos[2]);
      T add = T(ndo[l]) / hd * bn;
      if (l == lface) add += rv;
      s_r[B] += add;
    }
  }
  __syncthreads();
}

template <typename T, int NP, int NQ>
__global__ __launch_bounds__(64) void poisson_kernel(const MeshDev M, const T* __restrict__ p, T* __restrict__ y) {
  using Sh = PoiShape<T, NP, NQ>;
  constexpr TabLayout L = tab_layout(NP, NQ, NQ);
  constexpr int NP3 = Sh::NP3, NPTS = Sh::NPTS;
  __shared__ T s_p[NP3];
  __shared__ T s_r[NP3];
  __shared__ T s_big[Sh::BIG];
  const int tid = threadIdx.x, nt = blockDim.x;
  const int64_t e = blockIdx.x;
  const int ex = (int)(e % M.nx), ey = (int)((e / M.nx) % M.ny), ez = (int)(e / ((int64_t)M.nx * M.ny));
  const T hx = T(M.hx), hz = T(M.hz), hy = T(M.hy[ey]);
  const double* Sq = M.tab + L.S;
  const double* Dq = M.tab + L.D;
  const double* wq = M.tab + L.w;

  for (int i = tid; i < NP3; i += nt) s_p[i] = p[e * NP3 + i];
  __syncthreads();
  T* s_val = s_big;
  T* s_grad = s_big + NPTS;  // [d][pt]
  {
    T* tA = s_grad;
    T* tB = tA + NQ * NP * NP;
    sweep<0, NP, NP, NP, NQ, false, false>(s_p, NP3, tA, 0, Sq, T(1), 1);
    __syncthreads();
    sweep<1, NQ, NP, NP, NQ, false, false>(tA, 0, tB, 0, Sq, T(1), 1);
    __syncthreads();
    sweep<2, NQ, NQ, NP, NQ, false, false>(tB, 0, s_val, 0, Sq, T(1), 1);
    __syncthreads();
  }
  const T vol = hx * hy * hz;
  sweep<0, NQ, NQ, NQ, NQ, false, false>(s_val, 0, s_grad + 0 * NPTS, 0, Dq, T(1) / hx, 1);
  sweep<1, NQ, NQ, NQ, NQ, false, false>(s_val, 0, s_grad + 1 * NPTS, 0, Dq, T(1) / hy, 1);
  sweep<2, NQ, NQ, NQ, NQ, false, false>(s_val, 0, s_grad + 2 * NPTS, 0, Dq, T(1) / hz, 1);
  __syncthreads();
  for (int pt = tid; pt < NPTS; pt += nt) {
    const int qx = pt % NQ, qy = (pt / NQ) % NQ, qz = pt / (NQ * NQ);
    const T w = T(wq[qx]) * T(wq[qy]) * T(wq[qz]) * vol;
#pragma unroll
    for (int d = 0; d < 3; ++d) s_grad[d * NPTS + pt] *= w;
  }
  __syncthreads();
  sweep<0, NQ, NQ, NQ, NQ, true, false>(s_grad + 0 * NPTS, 0, s_val, 0, Dq, T(1) / hx, 1);
  __syncthreads();
  sweep<1, NQ, NQ, NQ, NQ, true, true>(s_grad + 1 * NPTS, 0, s_val, 0, Dq, T(1) / hy, 1);
  __syncthreads();
  sweep<2, NQ, NQ, NQ, NQ, true, true>(s_grad + 2 * NPTS, 0, s_val, 0, Dq, T(1) / hz, 1);
  __syncthreads();
  {
    T* tB = s_grad;
    T* tA = tB + NQ * NQ * NP;
    sweep<2, NQ, NQ, NQ, NP, true, false>(s_val, 0, tB, 0, Sq, T(1), 1);
    __syncthreads();
    sweep<1, NQ, NQ, NP, NP, true, false>(tB, 0, tA, 0, Sq, T(1), 1);
    __syncthreads();
    sweep<0, NQ, NP, NP, NP, true, false>(tA, 0, s_r, 0, Sq, T(1), 1);
    __syncthreads();
  }
  poi_face<T, NP, NQ, 0, 0>(M, p, s_p, s_r, s_big, ex, ey, ez, hx, hy, hz);
  poi_face<T, NP, NQ, 0, 1>(M, p, s_p, s_r, s_big, ex, ey, ez, hx, hy, hz);
  poi_face<T, NP, NQ, 1, 0>(M, p, s_p, s_r, s_big, ex, ey, ez, hx, hy, hz);
  poi_face<T, NP, NQ, 1, 1>(M, p, s_p, s_r, s_big, ex, ey, ez, hx, hy, hz);
  poi_face<T, NP, NQ, 2, 0>(M, p, s_p, s_r, s_big, ex, ey, ez, hx, hy, hz);
  poi_face<T, NP, NQ, 2, 1>(M, p, s_p, s_r, s_big, ex, ey, ez, hx, hy, hz);
  for (int i = tid; i < NP3; i += nt) y[e * NP3 + i] = s_r[i];
}

// Diagonal of A for box cells.  The basis is a tensor product, so every term
// separates into 1-D integrals: with M_i = int N_i^2, K_i = int N_i'^2 (Gauss
// rule of the operator, exact), the cell term is
//   |J| (K_i/hx^2 M_j M_m + M_i K_j/hy^2 M_m + M_i M_j K_m/hz^2)
// and an interior face in direction d at xi_d = s contributes
//   |F| M_t1 M_t2 [ tau (N_i(s) - P)N_i(s) - N_i(s) sg (N_i'(s) + P')/(2 h)
//                   - sg N_i'(s)/(2 h) (N_i(s) - P) ]
// where P, P' are the trace of the same basis function seen from the
// neighbour, non-zero only when the cell is its own periodic neighbour.
template <int NP, int NQ>
__global__ void poisson_diag_kernel(const MeshDev M, int64_t ncell, double* __restrict__ dg, float* __restrict__ dg32) {
  constexpr TabLayout L = tab_layout(NP, NQ, NQ);
  constexpr int NP3 = NP * NP * NP;
  const int64_t gid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (gid >= ncell * NP3) return;
  const int64_t e = gid / NP3;
  const int B = (int)(gid - e * NP3);
  const int idx[3] = {B % NP, (B / NP) % NP, B / (NP * NP)};
  const int ce[3] = {(int)(e % M.nx), (int)((e / M.nx) % M.ny), (int)(e / ((int64_t)M.nx * M.ny))};
  const double h[3] = {M.hx, M.hy[ce[1]], M.hz};
  const double* S = M.tab + L.S;
  const double* Sd = M.tab + L.Sd;
  const double* w = M.tab + L.w;
  double Mi[3], Ki[3];
  for (int a = 0; a < 3; ++a) {
    double m = 0, k = 0;
    for (int q = 0; q < NQ; ++q) {
      const double s = S[q * NP + idx[a]], sd = Sd[q * NP + idx[a]];
      m += w[q] * s * s;
      k += w[q] * sd * sd;
    }
    Mi[a] = m;
    Ki[a] = k;
  }
  const double vol = h[0] * h[1] * h[2];
  double acc = vol * (Ki[0] / (h[0] * h[0]) * Mi[1] * Mi[2] + Mi[0] * Ki[1] / (h[1] * h[1]) * Mi[2] +
                      Mi[0] * Mi[1] * Ki[2] / (h[2] * h[2]));
  const int nmax[3] = {M.nx, M.ny, M.nz};
  for (int d = 0; d < 3; ++d) {
    const int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
    for (int s = 0; s < 2; ++s) {
      int j = ce[d] + (s ? 1 : -1);
      if (j < 0 || j >= nmax[d]) {
        if (d == 1 && !M.fully_periodic) continue;
        j = (j + nmax[d]) % nmax[d];
      }
      const bool self = (j == ce[d]);
      const double hn = (d == 1) ? M.hy[j] : h[d];
      const double tau = M.pen * fmax(1.0 / h[d], 1.0 / hn);
      const double sg = s ? 1.0 : -1.0;
      const double* nd = M.tab + (s ? L.nd1 : L.nd0);
      const double* ndo = M.tab + (s ? L.nd0 : L.nd1);
      const double Ns = (idx[d] == (s ? NP - 1 : 0)) ? 1.0 : 0.0;
      const double dNs = nd[idx[d]] / h[d];
      const double P = self ? ((idx[d] == (s ? 0 : NP - 1)) ? 1.0 : 0.0) : 0.0;
      const double dP = self ? ndo[idx[d]] / hn : 0.0;
      const double area = h[t1] * h[t2];
      const double jump = Ns - P;
      const double term = tau * jump * Ns - Ns * sg * 0.5 * (dNs + dP) - sg * 0.5 * dNs * jump;
      acc += area * Mi[t1] * Mi[t2] * term;
    }
  }
  dg[gid] = acc;
  dg32[gid] = (float)acc;
}

MeshDev make_meshdev_p(const dg_mesh* m) {
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
  M.tab = m->tab_p;
  M.pen = m->P.ip_factor_p * (m->P.k_p + 1.0) * (m->P.k_p + 1.0);
  return M;
}

}  // namespace

#define DG_POI_COMBOS(X) X(2, 2) X(3, 3) X(4, 4) X(5, 5) X(6, 6)

bool poisson_supported(int np, int nq) {
#define X(a, b) \
  if (np == a && nq == b) return true;
  DG_POI_COMBOS(X)
#undef X
  return false;
}

const char* poisson_combos() { return "poisson (k+1, nq_p): (2,2) (3,3) (4,4) (5,5) (6,6)"; }

int launch_poisson(const dg_mesh* m, dg_prec prec, const void* p, void* y, hipStream_t s) {
  const MeshDev M = make_meshdev_p(m);
  const unsigned nb = (unsigned)m->ncell;
#define X(a, b)                                                                                           \
  if (m->np_p == a && m->P.nq_p == b) {                                                                   \
    if (prec == DG_F64)                                                                                   \
      hipLaunchKernelGGL((poisson_kernel<double, a, b>), dim3(nb), dim3(64), 0, s, M,                     \
                         static_cast<const double*>(p), static_cast<double*>(y));                         \
    else                                                                                                  \
      hipLaunchKernelGGL((poisson_kernel<float, a, b>), dim3(nb), dim3(64), 0, s, M,                      \
                         static_cast<const float*>(p), static_cast<float*>(y));                           \
    return check_hip(hipGetLastError(), "poisson kernel launch");                                         \
  }
  DG_POI_COMBOS(X)
#undef X
  return set_error(DG_ERR_UNSUPPORTED, "poisson degree/quadrature combination not compiled");
}

int launch_poisson_diag(const dg_mesh* m, hipStream_t s) {
  const MeshDev M = make_meshdev_p(m);
  const int64_t n = m->n_p;
  const unsigned nb = (unsigned)((n + 255) / 256);
#define X(a, b)                                                                                           \
  if (m->np_p == a && m->P.nq_p == b) {                                                                   \
    hipLaunchKernelGGL((poisson_diag_kernel<a, b>), dim3(nb), dim3(256), 0, s, M, m->ncell, m->diag,      \
                       m->diag32);                                                                        \
    return check_hip(hipGetLastError(), "poisson diagonal launch");                                       \
  }
  DG_POI_COMBOS(X)
#undef X
  return set_error(DG_ERR_UNSUPPORTED, "poisson degree/quadrature combination not compiled");
}

}  // namespace dgwm
