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
  static constexpr int NL = 6 * 2 * NP2;   // neighbour layers [face][val|d_n][NP2]
  static constexpr int OL = 6 * 2 * NP2;   // own layers
  static constexpr int FL = 6 * 2 * FP;    // fluxes [face][q-test | d_n q-test][pt]
  static constexpr int RB = 6 * 2 * NP2;   // integrated face tests [face][value | normal][NP2]
  static constexpr int FACE = NL + OL + FL + RB;
  static constexpr int VOL = 4 * NPTS;
  static constexpr int BIG = VOL > FACE ? VOL : FACE;
};

// node index base + l * stride of the line along direction D through (a, b)
template <int NP>
__device__ __forceinline__ void poi_line(int D, int a, int b, int& base, int& stride) {
  if (D == 0) {
    base = NP * (a + NP * b);
    stride = 1;
  } else if (D == 1) {
    base = a + NP * NP * b;
    stride = NP;
  } else {
    base = a + NP * b;
    stride = NP * NP;
  }
}

// neighbour across face (D, S): -1 for a (Neumann) wall
__device__ __forceinline__ int64_t poi_nb(const MeshDev& M, int ex, int ey, int ez, int D, int S, int& ny1) {
  int n[3] = {ex, ey, ez};
  const int nmax = D == 0 ? M.nx : (D == 1 ? M.ny : M.nz);
  int j = n[D] + (S ? 1 : -1);
  if (j < 0 || j >= nmax) {
    if (D == 1 && !M.fully_periodic) return -1;
    j = (j + nmax) % nmax;
  }
  n[D] = j;
  ny1 = n[1];
  return n[0] + (int64_t)M.nx * (n[1] + (int64_t)M.ny * n[2]);
}

template <typename T, int NP, int NQ>
__global__ __launch_bounds__(64) void poisson_kernel(const MeshDev M, const T* __restrict__ p, T* __restrict__ y) {
  using Sh = PoiShape<T, NP, NQ>;
  constexpr TabLayout L = tab_layout(NP, NQ, NQ);
  constexpr int NP2 = Sh::NP2, NP3 = Sh::NP3, NPTS = Sh::NPTS, FP = Sh::FP;
  __shared__ T s_p[NP3];
  __shared__ T s_r[NP3];
  __shared__ T s_nl[Sh::NL];
  __shared__ T s_big[Sh::BIG];
  __shared__ T s_ft[NQ * NP + NQ + 2 * NP];  // S, w, N'(0), N'(1) for the face phases
  const int tid = threadIdx.x, nt = blockDim.x;
  const int64_t e = blockIdx.x;
  const int ex = (int)(e % M.nx), ey = (int)((e / M.nx) % M.ny), ez = (int)(e / ((int64_t)M.nx * M.ny));
  const T hx = T(M.hx), hz = T(M.hz), hy = T(M.hy[ey]);
  auto hdir = [&](int d) { return d == 0 ? hx : (d == 1 ? hy : hz); };
  const double* Sq = M.tab + L.S;  // volume sweeps: uniform indices, scalar cache
  const double* Dq = M.tab + L.D;
  const double* wq = M.tab + L.w;
  const double* nd0 = M.tab + L.nd0;
  const double* nd1 = M.tab + L.nd1;

  // own values, face tables, and the six neighbour face layers (value, normal derivative)
  for (int i = tid; i < NP3; i += nt) s_p[i] = p[e * NP3 + i];
  for (int i = tid; i < NQ * NP + NQ + 2 * NP; i += nt) {
    const int o = i < NQ * NP ? L.S + i : (i < NQ * NP + NQ ? L.w + i - NQ * NP : L.nd0 + i - NQ * NP - NQ);
    s_ft[i] = T(M.tab[o]);
  }
  for (int t = tid; t < 6 * NP2; t += nt) {
    const int f = t / NP2, k = t - f * NP2;
    const int D = f >> 1, S = f & 1;
    int ny1 = 0;
    const int64_t nb = poi_nb(M, ex, ey, ez, D, S, ny1);
    T val = 0, der = 0;
    if (nb >= 0) {
      int base, stride;
      poi_line<NP>(D, k % NP, k / NP, base, stride);
      const T* src = p + nb * NP3 + base;
      const double* nd = S ? nd0 : nd1;  // neighbour's face is at xi_D = 1 - S
      T x[NP];
#pragma unroll
      for (int l = 0; l < NP; ++l) x[l] = src[l * stride];
#pragma unroll
      for (int l = 0; l < NP; ++l) der += T(nd[l]) * x[l];
      val = x[S ? 0 : NP - 1];
      const T hdn = D == 1 ? T(M.hy[ny1]) : hdir(D);
      der /= hdn;
    }
    s_nl[(f * 2 + 0) * NP2 + k] = val;
    s_nl[(f * 2 + 1) * NP2 + k] = der;
  }
  __syncthreads();

  // volume term: (grad q, grad p) by sum factorization
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

  // face terms of all six faces (tables from LDS: their indices vary across lanes)
  const T* fS = s_ft;
  const T* fw = s_ft + NQ * NP;
  const T* fnd0 = fw + NQ;
  const T* fnd1 = fnd0 + NP;
  T* ol = s_big;              // own layers [face][val|d_n][NP2]
  T* fl = ol + Sh::OL;        // fluxes [face][2][FP]
  T* rb = fl + Sh::FL;        // [face][value test | normal test][NP2]
  for (int t = tid; t < 6 * NP2; t += nt) {
    const int f = t / NP2, k = t - f * NP2;
    const int D = f >> 1, S = f & 1;
    int base, stride;
    poi_line<NP>(D, k % NP, k / NP, base, stride);
    const T* nd = S ? fnd1 : fnd0;
    T der = 0;
#pragma unroll
    for (int l = 0; l < NP; ++l) der += T(nd[l]) * s_p[base + l * stride];
    ol[(f * 2 + 0) * NP2 + k] = s_p[base + (S ? NP - 1 : 0) * stride];
    ol[(f * 2 + 1) * NP2 + k] = der / hdir(D);
  }
  __syncthreads();
  // traces of both sides at the face Gauss points, then the SIP flux
  for (int t = tid; t < 6 * FP; t += nt) {
    const int f = t / FP, pt = t - f * FP;
    const int D = f >> 1, S = f & 1;
    int ny1 = 0;
    if (poi_nb(M, ex, ey, ez, D, S, ny1) < 0) {
      fl[(f * 2 + 0) * FP + pt] = 0;
      fl[(f * 2 + 1) * FP + pt] = 0;
      continue;
    }
    const int q1 = pt % NQ, q2 = pt / NQ;
    const T* lo = ol + f * 2 * NP2;
    const T* ln = s_nl + f * 2 * NP2;
    T vm = 0, dm = 0, vp = 0, dp = 0;
#pragma unroll
    for (int i2 = 0; i2 < NP; ++i2) {
      T a0 = 0, a1 = 0, a2 = 0, a3 = 0;
#pragma unroll
      for (int i1 = 0; i1 < NP; ++i1) {
        const T s1 = (fS[q1 * NP + i1]);
        a0 += s1 * lo[i1 + NP * i2];
        a1 += s1 * lo[NP2 + i1 + NP * i2];
        a2 += s1 * ln[i1 + NP * i2];
        a3 += s1 * ln[NP2 + i1 + NP * i2];
      }
      const T s2 = (fS[q2 * NP + i2]);
      vm += s2 * a0;
      dm += s2 * a1;
      vp += s2 * a2;
      dp += s2 * a3;
    }
    const int T1 = D == 0 ? 1 : 0, T2 = D == 2 ? 1 : 2;
    const T ht1 = hdir(T1), ht2 = hdir(T2), hd = hdir(D);
    const T hdn = D == 1 ? T(M.hy[ny1]) : hd;
    const T tauF = T(M.pen) * (T(1) / hd > T(1) / hdn ? T(1) / hd : T(1) / hdn);
    const T sg = S ? T(1) : T(-1);
    const T wf = (fw[q1]) * (fw[q2]) * ht1 * ht2;
    const T jmp = vm - vp;
    const T avg_n = T(0.5) * (dm + dp) * sg;
    fl[(f * 2 + 0) * FP + pt] = wf * (-avg_n + tauF * jmp);      // tested with q
    fl[(f * 2 + 1) * FP + pt] = wf * (T(-0.5) * jmp * sg);       // tested with d q / d x_D
  }
  __syncthreads();
  // integrate against the face traces of the test functions
  for (int t = tid; t < 6 * NP2; t += nt) {
    const int f = t / NP2, k = t - f * NP2;
    const int i1 = k % NP, i2 = k / NP;
    const T* a = fl + f * 2 * FP;
    T rv = 0, bn = 0;
#pragma unroll
    for (int q2 = 0; q2 < NQ; ++q2) {
      T a0 = 0, a1 = 0;
#pragma unroll
      for (int q1 = 0; q1 < NQ; ++q1) {
        const T s1 = (fS[q1 * NP + i1]);
        a0 += s1 * a[q1 + NQ * q2];
        a1 += s1 * a[FP + q1 + NQ * q2];
      }
      rv += (fS[q2 * NP + i2]) * a0;
      bn += (fS[q2 * NP + i2]) * a1;
    }
    rb[(f * 2 + 0) * NP2 + k] = rv;
    rb[(f * 2 + 1) * NP2 + k] = bn / hdir(f >> 1);
  }
  __syncthreads();
  // scatter: every node gathers the contributions of the six faces
  for (int B = tid; B < NP3; B += nt) {
    const int ii[3] = {B % NP, (B / NP) % NP, B / NP2};
    T acc = s_r[B];
#pragma unroll
    for (int D = 0; D < 3; ++D) {
      const int a = D == 0 ? ii[1] : ii[0];
      const int b = D == 2 ? ii[1] : ii[2];
      const int k = a + NP * b;
      const int l = ii[D];
      acc += (fnd0[l]) * rb[((2 * D + 0) * 2 + 1) * NP2 + k] + (fnd1[l]) * rb[((2 * D + 1) * 2 + 1) * NP2 + k];
      if (l == 0) acc += rb[((2 * D + 0) * 2 + 0) * NP2 + k];
      if (l == NP - 1) acc += rb[((2 * D + 1) * 2 + 0) * NP2 + k];
    }
    y[e * NP3 + B] = acc;
  }
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
