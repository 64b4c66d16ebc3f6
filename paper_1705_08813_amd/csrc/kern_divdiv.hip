// Div-div penalty of the projection step (arXiv 1705.08813, Sec. 4.2, eqs.
// div-div and tauD), FP64, flat (box) meshes.
//
//   tau_D,e = ||u||_e h_e dt/Cr,   ||u||_e = |Omega_e|^{-1} int_e |u| dOmega,  h_e = |Omega_e|^{1/3}
//   D(v, u) = (div v, tau_D,e div u)_e
//
// for every velocity test function v (N_B e_c, and in enriched cells psi e_c
// for l = 0 or psi N_B e_c with the eight trilinear vertex functions N_B for
// l = 1, Sec. 3.1 eq. enrichment), u the full velocity (its enrichment
// included), with the velocity
// quadrature of the cell (nq^3, nq x nqy x nq in enriched cells).  Both are
// cell-local: one workgroup per cell, sum-factorized sweeps with the 1-D
// tables as compile-time literals (the three components' sweeps of a phase
// run on separate wavefronts), no faces.
#include "ctab.h"
#include "kern_common.h"

namespace dgwm {

namespace {

constexpr int kDdThreads = 256;

struct DdArgs {
  int nx, ny, nz, lower_slot, nslots, psi_pts;
  int64_t ncell;
  double hx, hz, dt_over_cr;
  const double* hy;        // ny heights
  const double* psi;       // [enr][psi_pts][4]
  const double* u;
  const double* tau_d;     // [cell] (apply)
  double* out;             // tau_d [cell] (tau kernel) or D u (velocity layout)
};

// Trilinear vertex function B (B = bx + 2 (by + 2 bz)) at reference point x
// and its reference derivatives d[3].
__device__ __forceinline__ double dd_vtx(int B, const double x[3], double d[3]) {
  const double a0 = (B & 1) ? x[0] : 1.0 - x[0], a1 = (B & 2) ? x[1] : 1.0 - x[1], a2 = (B & 4) ? x[2] : 1.0 - x[2];
  d[0] = ((B & 1) ? 1.0 : -1.0) * a1 * a2;
  d[1] = a0 * ((B & 2) ? 1.0 : -1.0) * a2;
  d[2] = a0 * a1 * ((B & 4) ? 1.0 : -1.0);
  return a0 * a1 * a2;
}

template <int NP, int NQ>
using MS = ct::MatS<NP, NQ>;
template <int NP, int NQ>
using MD = ct::MatSd<NP, NQ>;

// Cell of block b: regular cells b = ex + nx (ly + nlayers ez), ey = layer_lo
// + ly; enriched cells b = enriched index.
template <bool ENR>
__device__ __forceinline__ int64_t dd_cell(const DdArgs& A, int64_t b, int layer_lo, int nlayers, int& ey) {
  const int ex = (int)(b % A.nx);
  const int64_t t0 = b / A.nx;
  int64_t ez;
  if (ENR) {
    const int slot = (int)(t0 % A.nslots);
    ez = t0 / A.nslots;
    ey = slot == A.lower_slot ? 0 : A.ny - 1;
  } else {
    ey = layer_lo + (int)(t0 % nlayers);
    ez = t0 / nlayers;
  }
  return ex + (int64_t)A.nx * (ey + (int64_t)A.ny * ez);
}

// Fixed-order block sum of NV values per thread (every thread gets the sums).
template <int NV>
__device__ __forceinline__ void dd_block_sum(double (&v)[NV], double* red, int tid) {
  constexpr int NW = kDdThreads / 64;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1)
#pragma unroll
    for (int i = 0; i < NV; ++i) v[i] += __shfl_down(v[i], off, 64);
  if ((tid & 63) == 0)
#pragma unroll
    for (int i = 0; i < NV; ++i) red[i * NW + (tid >> 6)] = v[i];
  __syncthreads();
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    v[i] = 0.0;
    for (int w = 0; w < NW; ++w) v[i] += red[i * NW + w];
  }
}

template <int NP, int NQ, int NQY, bool ENR, int LE>
__global__ __launch_bounds__(kDdThreads) void divdiv_tau_kernel(const DdArgs A, int layer_lo, int nlayers) {
  constexpr int NP3 = NP * NP * NP, NPT = NQ * NQY * NQ;
  constexpr auto& tq = ct::tab<NP, NQ>;
  constexpr auto& ty = ct::tab<NP, NQY>;
  __shared__ double su[3 * NP3];
  __shared__ double w0[3 * NPT], w1[3 * NPT];
  __shared__ double ut[3 * LE];
  __shared__ double red[kDdThreads / 64];
  const int tid = threadIdx.x;
  int ey;
  const int64_t b = blockIdx.x;
  const int64_t e = dd_cell<ENR>(A, b, layer_lo, nlayers, ey);
  const double* ue = A.u + e * 3 * NP3;
  for (int i = tid; i < 3 * NP3; i += kDdThreads) su[i] = ue[i];
  if (ENR && tid < 3 * LE) ut[tid] = A.u[A.ncell * 3 * NP3 + b * 3 * LE + tid];
  __syncthreads();
  sweep_c<0, NP, NP, NP, NQ, false, false, MS<NP, NQ>>(su, NP3, w0, NPT, 1.0, 3);
  __syncthreads();
  sweep_c<1, NQ, NP, NP, NQY, false, false, MS<NP, NQY>>(w0, NPT, w1, NPT, 1.0, 3);
  __syncthreads();
  sweep_c<2, NQ, NQY, NP, NQ, false, false, MS<NP, NQ>>(w1, NPT, w0, NPT, 1.0, 3);
  __syncthreads();
  double v[1] = {0.0};
  for (int q = tid; q < NPT; q += kDdThreads) {
    const int qx = q % NQ, qy = (q / NQ) % NQY, qz = q / (NQ * NQY);
    double a = w0[q], bb = w0[NPT + q], c = w0[2 * NPT + q];
    if (ENR) {
      const double ps = A.psi[(b * A.psi_pts + q) * 4];
      double L[3] = {ut[0], ut[LE], ut[2 * LE]};  // the enrichment weights at the point
      if (LE == 8) {
        const double x[3] = {tq.g[qx], ty.g[qy], tq.g[qz]};
        L[0] = L[1] = L[2] = 0.0;
#pragma unroll
        for (int B = 0; B < 8; ++B) {
          double dv[3];
          const double nb = dd_vtx(B, x, dv);
#pragma unroll
          for (int cc = 0; cc < 3; ++cc) L[cc] += nb * ut[cc * LE + B];
        }
      }
      a += ps * L[0];
      bb += ps * L[1];
      c += ps * L[2];
    }
    v[0] += tq.w[qx] * ty.w[qy] * tq.w[qz] * sqrt(a * a + bb * bb + c * c);
  }
  dd_block_sum<1>(v, red, tid);
  if (tid == 0) {
    // reference weights sum to 1: the volume average of |u| is v[0] itself
    const double vol = A.hx * A.hy[ey] * A.hz;
    A.out[e] = v[0] * cbrt(vol) * A.dt_over_cr;
  }
}

template <int NP, int NQ, int NQY, bool ENR, int LE>
__global__ __launch_bounds__(kDdThreads) void divdiv_apply_kernel(const DdArgs A, int layer_lo, int nlayers) {
  constexpr int NP3 = NP * NP * NP, NPT = NQ * NQY * NQ;
  constexpr auto& tq = ct::tab<NP, NQ>;
  constexpr auto& ty = ct::tab<NP, NQY>;
  __shared__ double su[3 * NP3];
  __shared__ double w0[3 * NPT], w1[3 * NPT];
  __shared__ double ut[3 * LE];
  __shared__ double red[3 * LE * (kDdThreads / 64)];
  const int tid = threadIdx.x;
  int ey;
  const int64_t b = blockIdx.x;
  const int64_t e = dd_cell<ENR>(A, b, layer_lo, nlayers, ey);
  const double* ue = A.u + e * 3 * NP3;
  for (int i = tid; i < 3 * NP3; i += kDdThreads) su[i] = ue[i];
  if (ENR && tid < 3 * LE) ut[tid] = A.u[A.ncell * 3 * NP3 + b * 3 * LE + tid];
  __syncthreads();
  const double h[3] = {A.hx, A.hy[ey], A.hz};
  // d_c u_c at the points: component c takes the derivative table along c
  sweep_c<0, NP, NP, NP, NQ, false, false, MD<NP, NQ>>(su, NP3, w0, NPT, 1.0, 1, 0);
  sweep_c<0, NP, NP, NP, NQ, false, false, MS<NP, NQ>>(su + NP3, NP3, w0 + NPT, NPT, 1.0, 1, 64);
  sweep_c<0, NP, NP, NP, NQ, false, false, MS<NP, NQ>>(su + 2 * NP3, NP3, w0 + 2 * NPT, NPT, 1.0, 1, 128);
  __syncthreads();
  sweep_c<1, NQ, NP, NP, NQY, false, false, MS<NP, NQY>>(w0, NPT, w1, NPT, 1.0, 1, 0);
  sweep_c<1, NQ, NP, NP, NQY, false, false, MD<NP, NQY>>(w0 + NPT, NPT, w1 + NPT, NPT, 1.0, 1, 64);
  sweep_c<1, NQ, NP, NP, NQY, false, false, MS<NP, NQY>>(w0 + 2 * NPT, NPT, w1 + 2 * NPT, NPT, 1.0, 1, 128);
  __syncthreads();
  sweep_c<2, NQ, NQY, NP, NQ, false, false, MS<NP, NQ>>(w1, NPT, w0, NPT, 1.0, 1, 0);
  sweep_c<2, NQ, NQY, NP, NQ, false, false, MS<NP, NQ>>(w1 + NPT, NPT, w0 + NPT, NPT, 1.0, 1, 64);
  sweep_c<2, NQ, NQY, NP, NQ, false, false, MD<NP, NQ>>(w1 + 2 * NPT, NPT, w0 + 2 * NPT, NPT, 1.0, 1, 128);
  __syncthreads();
  // f = w |J| tau_D div u; tested with d_c N_B = (1/h_c) d/dxi_c and, in enriched cells, d_c phi for the
  // enrichment functions phi = psi (l = 0) or psi N_B (l = 1): d_c phi = N_B d_c psi + psi d_c N_B
  const double scale = h[0] * h[1] * h[2] * A.tau_d[e];
  double ve[3 * LE];
#pragma unroll
  for (int i = 0; i < 3 * LE; ++i) ve[i] = 0.0;
  for (int q = tid; q < NPT; q += kDdThreads) {
    const int qx = q % NQ, qy = (q / NQ) % NQY, qz = q / (NQ * NQY);
    double dv = w0[q] / h[0] + w0[NPT + q] / h[1] + w0[2 * NPT + q] / h[2];
    const double* ps = ENR ? A.psi + (b * A.psi_pts + q) * 4 : nullptr;
    double gphi[LE][3];  // physical gradients of the enrichment functions at the point
    if (ENR) {
      if (LE == 1) {
#pragma unroll
        for (int c = 0; c < 3; ++c) gphi[0][c] = ps[1 + c];
      } else {
        const double x[3] = {tq.g[qx], ty.g[qy], tq.g[qz]};
#pragma unroll
        for (int B = 0; B < LE; ++B) {
          double d[3];
          const double nb = dd_vtx(B, x, d);
#pragma unroll
          for (int c = 0; c < 3; ++c) gphi[B][c] = nb * ps[1 + c] + ps[0] * d[c] / h[c];
        }
      }
#pragma unroll
      for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int B = 0; B < LE; ++B) dv += gphi[B][c] * ut[c * LE + B];
    }
    const double f = tq.w[qx] * ty.w[qy] * tq.w[qz] * scale * dv;
    if (ENR) {
#pragma unroll
      for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int B = 0; B < LE; ++B) ve[c * LE + B] += gphi[B][c] * f;
    }
    w1[q] = f / h[0];
    w1[NPT + q] = f / h[1];
    w1[2 * NPT + q] = f / h[2];
  }
  __syncthreads();
  sweep_c<0, NQ, NQY, NQ, NP, true, false, MD<NP, NQ>>(w1, NPT, w0, NPT, 1.0, 1, 0);
  sweep_c<0, NQ, NQY, NQ, NP, true, false, MS<NP, NQ>>(w1 + NPT, NPT, w0 + NPT, NPT, 1.0, 1, 64);
  sweep_c<0, NQ, NQY, NQ, NP, true, false, MS<NP, NQ>>(w1 + 2 * NPT, NPT, w0 + 2 * NPT, NPT, 1.0, 1, 128);
  __syncthreads();
  sweep_c<1, NP, NQY, NQ, NP, true, false, MS<NP, NQY>>(w0, NPT, w1, NPT, 1.0, 1, 0);
  sweep_c<1, NP, NQY, NQ, NP, true, false, MD<NP, NQY>>(w0 + NPT, NPT, w1 + NPT, NPT, 1.0, 1, 64);
  sweep_c<1, NP, NQY, NQ, NP, true, false, MS<NP, NQY>>(w0 + 2 * NPT, NPT, w1 + 2 * NPT, NPT, 1.0, 1, 128);
  __syncthreads();
  double* oe = A.out + e * 3 * NP3;
  sweep_c<2, NP, NP, NQ, NP, true, false, MS<NP, NQ>>(w1, NPT, oe, NP3, 1.0, 1, 0);
  sweep_c<2, NP, NP, NQ, NP, true, false, MS<NP, NQ>>(w1 + NPT, NPT, oe + NP3, NP3, 1.0, 1, 64);
  sweep_c<2, NP, NP, NQ, NP, true, false, MD<NP, NQ>>(w1 + 2 * NPT, NPT, oe + 2 * NP3, NP3, 1.0, 1, 128);
  if (ENR) {
    dd_block_sum<3 * LE>(ve, red, tid);
    if (tid < 3 * LE) {
      double o = 0.0;  // (ve[tid] with a constant index, so ve stays in registers)
#pragma unroll
      for (int i = 0; i < 3 * LE; ++i) o = i == tid ? ve[i] : o;
      A.out[A.ncell * 3 * NP3 + b * 3 * LE + tid] = o;
    }
  }
}

}  // namespace

#define DG_DD_COMBOS(X) X(3, 4, 8) X(3, 4, 4) X(4, 4, 8) X(4, 5, 8) X(4, 5, 5) X(5, 7, 8) X(6, 8, 8)

int launch_divdiv(const dg_mesh* m, bool tau, const double* u, const double* tau_d, double dt_over_cr, double* out,
                  hipStream_t s) {
  if (m->curved) return launch_divdiv_curved(m, tau, u, tau_d, dt_over_cr, out, s);
  DdArgs A;
  A.nx = m->P.nx;
  A.ny = m->P.ny;
  A.nz = m->P.nz;
  A.lower_slot = m->lower_slot;
  A.nslots = m->n_enr_layers;
  A.psi_pts = m->psi_pts;
  A.ncell = m->ncell;
  A.hx = m->hx;
  A.hz = m->hz;
  A.dt_over_cr = dt_over_cr;
  A.hy = m->hy;
  A.psi = m->psi;
  A.u = u;
  A.tau_d = tau_d;
  A.out = out;
  const int lo = (m->P.fully_periodic || m->lower_slot < 0) ? 0 : 1;
  const int hi = (m->P.fully_periodic || m->upper_slot < 0) ? m->P.ny - 1 : m->P.ny - 2;
  const int nl = hi - lo + 1;
  const int64_t nreg = nl > 0 ? (int64_t)m->P.nx * nl * m->P.nz : 0;
  // without enriched cells only the regular kernels run and nq_wn is irrelevant
  const bool any_w = m->nenr == 0;
  const int nqw = m->P.nq_wn;
#define LAUNCH(KER, p, q, w, ENRV, LEV, grid, lo_, nl_) \
  hipLaunchKernelGGL((KER<p, q, w, ENRV, LEV>), dim3((unsigned)(grid)), dim3(kDdThreads), 0, s, A, lo_, nl_)
#define X(p, q, w)                                                                              \
  if (m->np_u == p && m->P.nq_u == q && (any_w || nqw == w)) {                                  \
    if (nreg > 0) {                                                                             \
      if (tau) LAUNCH(divdiv_tau_kernel, p, q, q, false, 1, nreg, lo, nl);                      \
      else LAUNCH(divdiv_apply_kernel, p, q, q, false, 1, nreg, lo, nl);                        \
      const int rc = check_hip(hipGetLastError(), "div-div kernel launch");                     \
      if (rc) return rc;                                                                        \
    }                                                                                           \
    if (m->nenr > 0) {                                                                          \
      if (m->nle == 8) {                                                                        \
        if (tau) LAUNCH(divdiv_tau_kernel, p, q, w, true, 8, m->nenr, 0, 0);                    \
        else LAUNCH(divdiv_apply_kernel, p, q, w, true, 8, m->nenr, 0, 0);                      \
      } else {                                                                                  \
        if (tau) LAUNCH(divdiv_tau_kernel, p, q, w, true, 1, m->nenr, 0, 0);                    \
        else LAUNCH(divdiv_apply_kernel, p, q, w, true, 1, m->nenr, 0, 0);                      \
      }                                                                                         \
    }                                                                                           \
    return check_hip(hipGetLastError(), "div-div kernel launch");                               \
  }
  DG_DD_COMBOS(X)
#undef X
#undef LAUNCH
  return set_error(DG_ERR_UNSUPPORTED, "div-div penalty: (k_u+1, nq_u, nq_wn) combination not compiled");
}

}  // namespace dgwm
