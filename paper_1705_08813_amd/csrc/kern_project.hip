// Cell-wise L2 projection onto the refreshed enriched space (arXiv
// 1705.08813, Sec. 3.2, eq. l2), FP64.
//
// After a wall-shear update the enrichment function of an enriched cell is
// psi_new instead of psi_old, and the velocity u_old = u_bar + psi_old u~ is
// carried over by  (v, u_new)_e = (v, u_old)_e  for every v of the new local
// space span{N_B} + span{psi_new} (per component), with the enriched cell's
// quadrature rule nq x nqy x nq.  Writing P for the L2 projection onto the
// polynomials of the cell, a = M^{-1} (N, psi) the coefficients of P psi and
// r = psi - P psi, the two-block system has the closed form
//   u~_new   = u~_old (r_new, r_old) / (r_new, r_new)
//   u_bar_new = u_bar_old + u~_old a_old - u~_new a_new
// (Schur complement on the enrichment row; (., .) the quadrature inner
// product).  A cell whose enrichment is switched off in the new space has
// psi_new = 0: then u~_new = 0 and u_bar_new = u_bar_old + u~_old a_old; a
// cell switched off in the old space has psi_old = 0, a_old = 0 and r_old = 0,
// so u_new = u_bar_old.  The residual functions r are formed pointwise before
// the inner products, which keeps the division well conditioned when psi is
// close to a polynomial (the mass matrix then has a condition number near
// 1e7, but (r, r) carries no cancellation).
//
// M is the tensor product of 1-D mass matrices (affine cells; |det J| cancels
// in a and in the ratio), so M^{-1} is three sweeps with the inverse 1-D
// matrices, and every other step is a sum-factorized sweep in LDS.  One
// workgroup per enriched cell; cells without enrichment are copied (or, in
// place, left alone).
#include "kern_common.h"

namespace dgwm {

namespace {

constexpr int kPrjThreads = 256;

struct ProjArgs {
  int nx, ny, nz, lower_slot, nslots, psi_pts;
  int64_t ncell;
  const double* tab;       // velocity tables (tab_layout(np, nq, nqy))
  const double* minv;      // [2][np][np]: inverse mass, x/z rule then wall-normal rule
  const double* psi_old;   // [enr][psi_pts][4]
  const double* psi_new;
  const int32_t* act_new;  // [enr]
  const double* u_old;
  double* u_new;            // may equal u_old
};

// out[c][...] = sum_l A[o][l] in[c][...] along one direction of a 3-D array
// stored with strides (1, E0, E0 E1); E = extents of `in`, MO = output extent
// along DIR; A is [MO][L] with row stride L (A^T when TR: A[l][o]).
template <int DIR, int E0, int E1, int E2, int MO, bool TR>
__device__ __forceinline__ void sweep2(const double* in, double* out, const double* A, int tid) {
  constexpr int L = DIR == 0 ? E0 : DIR == 1 ? E1 : E2;
  constexpr int O0 = DIR == 0 ? MO : E0, O1 = DIR == 1 ? MO : E1, O2 = DIR == 2 ? MO : E2;
  constexpr int NI = E0 * E1 * E2, NO = O0 * O1 * O2;
  for (int it = tid; it < 2 * NO; it += kPrjThreads) {
    const int c = it / NO, r = it - c * NO;
    const int o0 = r % O0, o1 = (r / O0) % O1, o2 = r / (O0 * O1);
    const int o = DIR == 0 ? o0 : DIR == 1 ? o1 : o2;
    const int base = (DIR == 0 ? 0 : o0) + E0 * ((DIR == 1 ? 0 : o1) + E1 * (DIR == 2 ? 0 : o2));
    constexpr int st = DIR == 0 ? 1 : DIR == 1 ? E0 : E0 * E1;
    const double* ip = in + c * NI + base;
    double s = 0.0;
#pragma unroll
    for (int l = 0; l < L; ++l) s += (TR ? A[l * MO + o] : A[o * L + l]) * ip[l * st];
    out[it] = s;
  }
}

template <int NP, int NQ, int NQY>
__global__ __launch_bounds__(kPrjThreads) void project_kernel(const ProjArgs A) {
  constexpr int NPT = NQ * NQY * NQ, NP3 = NP * NP * NP;
  constexpr TabLayout TL = tab_layout(NP, NQ, NQY);
  __shared__ double sS[NQ * NP], sSy[NQY * NP], sW[NQ], sWy[NQY], sMi[NP * NP], sMiy[NP * NP];
  __shared__ double ps[2 * NPT];        // psi (old, new) at the points, later r = psi - P psi
  __shared__ double f[2 * NPT];         // w_q psi
  __shared__ double t1[2 * NQ * NQY * NP];
  __shared__ double t2[2 * NQ * NP * NP];
  __shared__ double a[2 * NP3], b[2 * NP3];
  __shared__ double red[2 * (kPrjThreads / 64)];
  __shared__ double sut[3];                 // u~_old (read before any write: u_new may be u_old)
  const int tid = threadIdx.x;
  const int64_t enr = blockIdx.x;
  const int ex = (int)(enr % A.nx);
  const int64_t t0 = enr / A.nx;
  const int slot = (int)(t0 % A.nslots);
  const int ez = (int)(t0 / A.nslots);
  const int ey = slot == A.lower_slot ? 0 : A.ny - 1;
  const int64_t e = ex + (int64_t)A.nx * (ey + (int64_t)A.ny * ez);

  for (int i = tid; i < NQ * NP; i += kPrjThreads) sS[i] = A.tab[TL.S + i];
  for (int i = tid; i < NQY * NP; i += kPrjThreads) sSy[i] = A.tab[TL.Sy + i];
  for (int i = tid; i < NP * NP; i += kPrjThreads) {
    sMi[i] = A.minv[i];
    sMiy[i] = A.minv[NP * NP + i];
  }
  if (tid < NQ) sW[tid] = A.tab[TL.w + tid];
  if (tid < NQY) sWy[tid] = A.tab[TL.wy + tid];
  __syncthreads();
  // volume points q = qx + NQ (qy + NQY qz) are the first NPT entries of a cell's table
  const double* po = A.psi_old + enr * A.psi_pts * 4;
  const double* pn = A.psi_new + enr * A.psi_pts * 4;
  for (int q = tid; q < NPT; q += kPrjThreads) {
    const int qx = q % NQ, qy = (q / NQ) % NQY, qz = q / (NQ * NQY);
    const double w = sW[qx] * sWy[qy] * sW[qz];
    const double vo = po[q * 4], vn = pn[q * 4];
    ps[q] = vo;
    ps[NPT + q] = vn;
    f[q] = w * vo;
    f[NPT + q] = w * vn;
  }
  __syncthreads();
  // (N_B, psi) = S^T W psi, one sweep per direction
  sweep2<0, NQ, NQY, NQ, NP, true>(f, t1, sS, tid);     // [c][qz][qy][i]
  __syncthreads();
  sweep2<1, NP, NQY, NQ, NP, true>(t1, t2, sSy, tid);   // [c][qz][j][i]
  __syncthreads();
  sweep2<2, NP, NP, NQ, NP, true>(t2, a, sS, tid);      // [c][k][j][i]
  __syncthreads();
  // a = M^{-1} (N, psi) with M^{-1} = Mz^{-1} (x) My^{-1} (x) Mx^{-1}
  sweep2<0, NP, NP, NP, NP, false>(a, b, sMi, tid);
  __syncthreads();
  sweep2<1, NP, NP, NP, NP, false>(b, a, sMiy, tid);
  __syncthreads();
  sweep2<2, NP, NP, NP, NP, false>(a, b, sMi, tid);
  __syncthreads();
  // P psi at the points: interpolate b back
  sweep2<0, NP, NP, NP, NQ, false>(b, t2, sS, tid);     // [c][k][j][qx]
  __syncthreads();
  sweep2<1, NQ, NP, NP, NQY, false>(t2, t1, sSy, tid);  // [c][k][qy][qx]
  __syncthreads();
  sweep2<2, NQ, NQY, NP, NQ, false>(t1, f, sS, tid);    // [c][qz][qy][qx]
  __syncthreads();
  // r = psi - P psi, then (r_new, r_old) and (r_new, r_new)
  double num = 0.0, den = 0.0;
  for (int q = tid; q < NPT; q += kPrjThreads) {
    const int qx = q % NQ, qy = (q / NQ) % NQY, qz = q / (NQ * NQY);
    const double w = sW[qx] * sWy[qy] * sW[qz];
    const double ro = ps[q] - f[q], rn = ps[NPT + q] - f[NPT + q];
    num += w * rn * ro;
    den += w * rn * rn;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    num += __shfl_down(num, off, 64);
    den += __shfl_down(den, off, 64);
  }
  if ((tid & 63) == 0) {
    red[tid >> 6] = num;
    red[kPrjThreads / 64 + (tid >> 6)] = den;
  }
  const int64_t eo = A.ncell * 3 * NP3 + enr * 3;  // enrichment unknowns of the cell
  if (tid < 3) sut[tid] = A.u_old[eo + tid];
  __syncthreads();
  num = den = 0.0;
  for (int wv = 0; wv < kPrjThreads / 64; ++wv) {
    num += red[wv];
    den += red[kPrjThreads / 64 + wv];
  }
  const double ratio = (A.act_new[enr] && den > 0.0) ? num / den : 0.0;
  // each entry is read and written by the same thread, so u_new may alias u_old
  const double* ub = A.u_old + e * 3 * NP3;
  double* vb = A.u_new + e * 3 * NP3;
  for (int it = tid; it < 3 * NP3; it += kPrjThreads) {
    const int c = it / NP3, B = it - c * NP3;
    const double uto = sut[c];
    vb[it] = ub[it] + uto * b[B] - ratio * uto * b[NP3 + B];
  }
  if (tid < 3) A.u_new[eo + tid] = ratio * sut[tid];
}

}  // namespace

#define DG_PRJ_COMBOS(X) X(3, 4, 8) X(3, 4, 4) X(4, 4, 8) X(4, 5, 8) X(4, 5, 5) X(5, 7, 8) X(6, 8, 8)

int launch_project_velocity(const dg_mesh* m, const double* u_old, double* u_new, hipStream_t s) {
  if (u_new != u_old) {
    const int rc = check_hip(hipMemcpyAsync(u_new, u_old, sizeof(double) * m->n_vel, hipMemcpyDeviceToDevice, s),
                             "velocity copy");
    if (rc) return rc;
  }
  if (m->nenr == 0) return DG_OK;
  if (m->nenr > INT32_MAX) return set_error(DG_ERR_ARG, "projection: too many enriched cells");
  ProjArgs A;
  A.nx = m->P.nx;
  A.ny = m->P.ny;
  A.nz = m->P.nz;
  A.lower_slot = m->lower_slot;
  A.nslots = m->n_enr_layers;
  A.psi_pts = m->psi_pts;
  A.ncell = m->ncell;
  A.tab = m->tab_u;
  A.minv = m->minv;
  A.psi_old = m->psi_prev;
  A.psi_new = m->psi;
  A.act_new = m->act;
  A.u_old = u_old;
  A.u_new = u_new;
#define X(p, q, w)                                                                                  \
  if (m->np_u == p && m->P.nq_u == q && m->P.nq_wn == w) {                                          \
    hipLaunchKernelGGL((project_kernel<p, q, w>), dim3((unsigned)m->nenr), dim3(kPrjThreads), 0, s, A); \
    return check_hip(hipGetLastError(), "projection kernel launch");                                \
  }
  DG_PRJ_COMBOS(X)
#undef X
  return set_error(DG_ERR_UNSUPPORTED, "projection: (k_u+1, nq_u, nq_wn) combination not compiled");
}

}  // namespace dgwm
