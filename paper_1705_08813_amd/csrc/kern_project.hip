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
#include "ctab.h"
#include "kern_common.h"
#include "kern_tile.h"

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

// out[c][...] = sum_l A[o][l] in[c][...] along one direction of NC stacked
// 3-D arrays stored with strides (1, E0, E0 E1); E = extents of `in`, MO =
// output extent along DIR; A is [MO][L] with row stride L (A^T when TR:
// A[l][o]).  NT threads share the work.
template <int NC, int DIR, int E0, int E1, int E2, int MO, bool TR, int NT = kPrjThreads>
__device__ __forceinline__ void sweepn(const double* in, double* out, const double* A, int tid) {
  constexpr int L = DIR == 0 ? E0 : DIR == 1 ? E1 : E2;
  constexpr int O0 = DIR == 0 ? MO : E0, O1 = DIR == 1 ? MO : E1, O2 = DIR == 2 ? MO : E2;
  constexpr int NI = E0 * E1 * E2, NO = O0 * O1 * O2;
  for (int it = tid; it < NC * NO; it += NT) {
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

// 1-D tables of an enriched cell in LDS: S of the wall-parallel and of the
// wall-normal rule, their weights, the inverse 1-D mass matrices.
template <int NP, int NQ, int NQY>
struct Tab1d {
  double S[NQ * NP], Sy[NQY * NP], W[NQ], Wy[NQY], Mi[NP * NP], Miy[NP * NP];
};

template <int NP, int NQ, int NQY>
__device__ __forceinline__ void load_tab1d(const double* tab, const double* minv, Tab1d<NP, NQ, NQY>& T, int tid) {
  constexpr TabLayout TL = tab_layout(NP, NQ, NQY);
  for (int i = tid; i < NQ * NP; i += kPrjThreads) T.S[i] = tab[TL.S + i];
  for (int i = tid; i < NQY * NP; i += kPrjThreads) T.Sy[i] = tab[TL.Sy + i];
  for (int i = tid; i < NP * NP; i += kPrjThreads) {
    T.Mi[i] = minv[i];
    T.Miy[i] = minv[NP * NP + i];
  }
  if (tid < NQ) T.W[tid] = tab[TL.w + tid];
  if (tid < NQY) T.Wy[tid] = tab[TL.wy + tid];
}

// LDS work arrays of the polynomial part of NC <= 2 enrichment functions.
template <int NP, int NQ, int NQY>
struct PsiPoly {
  static constexpr int NPT = NQ * NQY * NQ, NP3 = NP * NP * NP;
  double r[2 * NPT];   // psi at the volume points, then r = psi - P psi
  double f[2 * NPT];
  double t1[2 * NQ * NQY * NP];
  double t2[2 * NQ * NP * NP];
  double a[2 * NP3];
  double b[2 * NP3];   // coefficients of P psi (nodal basis)
};

// For the NC tables psi[c] (entry 0 of [pt][4], volume points first, q = qx +
// NQ (qy + NQY qz)) of one cell: b[c] = K^{-1} (N, psi_c)_w, the nodal
// coefficients of the L2 projection P psi_c onto the cell's polynomials (K
// the weighted 1-D mass matrices' tensor product, |det J| cancels), and
// r[c] = psi_c - P psi_c at the points.  Ends with a barrier.
template <int NC, int NP, int NQ, int NQY, int PS = 4>
__device__ __forceinline__ void psi_poly_part(const double* const* psi, const Tab1d<NP, NQ, NQY>& T,
                                              PsiPoly<NP, NQ, NQY>& L, int tid, double* npsi_out = nullptr) {
  constexpr int NPT = NQ * NQY * NQ;
  for (int q = tid; q < NPT; q += kPrjThreads) {
    const int qx = q % NQ, qy = (q / NQ) % NQY, qz = q / (NQ * NQY);
    const double w = T.W[qx] * T.Wy[qy] * T.W[qz];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const double v = psi[c][q * PS];  // (PS: stride of the value table)
      L.r[c * NPT + q] = v;
      L.f[c * NPT + q] = w * v;
    }
  }
  __syncthreads();
  // (N_B, psi) = S^T W psi, one sweep per direction
  sweepn<NC, 0, NQ, NQY, NQ, NP, true>(L.f, L.t1, T.S, tid);     // [c][qz][qy][i]
  __syncthreads();
  sweepn<NC, 1, NP, NQY, NQ, NP, true>(L.t1, L.t2, T.Sy, tid);   // [c][qz][j][i]
  __syncthreads();
  sweepn<NC, 2, NP, NP, NQ, NP, true>(L.t2, L.a, T.S, tid);      // [c][k][j][i]
  __syncthreads();
  if (npsi_out)  // (N, psi_0)_w, before the inverse overwrites it
    for (int B = tid; B < NP * NP * NP; B += kPrjThreads) npsi_out[B] = L.a[B];
  // K^{-1} = Kz^{-1} (x) Ky^{-1} (x) Kx^{-1}
  sweepn<NC, 0, NP, NP, NP, NP, false>(L.a, L.b, T.Mi, tid);
  __syncthreads();
  sweepn<NC, 1, NP, NP, NP, NP, false>(L.b, L.a, T.Miy, tid);
  __syncthreads();
  sweepn<NC, 2, NP, NP, NP, NP, false>(L.a, L.b, T.Mi, tid);
  __syncthreads();
  // P psi at the points: interpolate b back
  sweepn<NC, 0, NP, NP, NP, NQ, false>(L.b, L.t2, T.S, tid);     // [c][k][j][qx]
  __syncthreads();
  sweepn<NC, 1, NQ, NP, NP, NQY, false>(L.t2, L.t1, T.Sy, tid);  // [c][k][qy][qx]
  __syncthreads();
  sweepn<NC, 2, NQ, NQY, NP, NQ, false>(L.t1, L.f, T.S, tid);    // [c][qz][qy][qx]
  __syncthreads();
  for (int q = tid; q < NC * NPT; q += kPrjThreads) L.r[q] -= L.f[q];
  __syncthreads();
}

// Block sum of NV values per thread (fixed order: lanes, then wavefronts).
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double* red, int tid) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1)
#pragma unroll
    for (int i = 0; i < NV; ++i) v[i] += __shfl_down(v[i], off, 64);
  constexpr int NW = kPrjThreads / 64;
  __syncthreads();
  if ((tid & 63) == 0)
#pragma unroll
    for (int i = 0; i < NV; ++i) red[i * NW + (tid >> 6)] = v[i];
  __syncthreads();
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    v[i] = 0.0;
    for (int wv = 0; wv < NW; ++wv) v[i] += red[i * NW + wv];
  }
}

__device__ __forceinline__ int64_t enriched_cell_index(int nx, int ny, int lower_slot, int nslots, int64_t enr) {
  const int ex = (int)(enr % nx);
  const int64_t t0 = enr / nx;
  const int slot = (int)(t0 % nslots);
  const int ez = (int)(t0 / nslots);
  const int ey = slot == lower_slot ? 0 : ny - 1;
  return ex + (int64_t)nx * (ey + (int64_t)ny * ez);
}

template <int NP, int NQ, int NQY>
__global__ __launch_bounds__(kPrjThreads) void project_kernel(const ProjArgs A) {
  constexpr int NPT = NQ * NQY * NQ, NP3 = NP * NP * NP;
  __shared__ Tab1d<NP, NQ, NQY> T;
  __shared__ PsiPoly<NP, NQ, NQY> L;
  __shared__ double red[2 * (kPrjThreads / 64)];
  __shared__ double sut[3];  // u~_old (read before any write: u_new may be u_old)
  const int tid = threadIdx.x;
  const int64_t enr = blockIdx.x;
  const int64_t e = enriched_cell_index(A.nx, A.ny, A.lower_slot, A.nslots, enr);
  load_tab1d<NP, NQ, NQY>(A.tab, A.minv, T, tid);
  __syncthreads();
  const double* psi[2] = {A.psi_old + enr * A.psi_pts * 4, A.psi_new + enr * A.psi_pts * 4};
  psi_poly_part<2, NP, NQ, NQY>(psi, T, L, tid);
  // (r_new, r_old) and (r_new, r_new)
  double v[2] = {0.0, 0.0};
  for (int q = tid; q < NPT; q += kPrjThreads) {
    const int qx = q % NQ, qy = (q / NQ) % NQY, qz = q / (NQ * NQY);
    const double w = T.W[qx] * T.Wy[qy] * T.W[qz];
    const double ro = L.r[q], rn = L.r[NPT + q];
    v[0] += w * rn * ro;
    v[1] += w * rn * rn;
  }
  const int64_t eo = A.ncell * 3 * NP3 + enr * 3;  // enrichment unknowns of the cell
  if (tid < 3) sut[tid] = A.u_old[eo + tid];
  block_sum<2>(v, red, tid);
  const double ratio = (A.act_new[enr] && v[1] > 0.0) ? v[0] / v[1] : 0.0;
  // each entry is read and written by the same thread, so u_new may alias u_old
  const double* ub = A.u_old + e * 3 * NP3;
  double* vb = A.u_new + e * 3 * NP3;
  for (int it = tid; it < 3 * NP3; it += kPrjThreads) {
    const int c = it / NP3, B = it - c * NP3;
    const double uto = sut[c];
    vb[it] = ub[it] + uto * L.b[B] - ratio * uto * L.b[NP3 + B];
  }
  if (tid < 3) A.u_new[eo + tid] = ratio * sut[tid];
}

// Degree-1 enrichment weights (Sec. 3.1 eq. enrichment, l = 1): the eight
// old and the eight new enrichment functions phi_B = psi N_B of the cell.
// With a_B = K^{-1} (N, phi_B)_w and r_B = phi_B - P phi_B for both sets,
// the new enrichment coefficients of each component solve
//   G_new u~_new = C u~_old,  G_new = (r_new, r_new)_w,  C = (r_new, r_old)_w,
// and u_bar_new = u_bar_old + sum_B u~_old,B a_old,B - sum_B u~_new,B a_new,B:
// the l = 0 closed form with the scalars replaced by 8 x 8 blocks.  A cell
// switched off in the new space gets u~_new = 0; one switched off in the old
// space has phi_old = 0, so a_old = 0, C = 0 and u_new = u_bar_old.
template <int NP, int NQ, int NQY>
__global__ __launch_bounds__(kPrjThreads) void project_l1_kernel(const ProjArgs A) {
  constexpr int NPT = NQ * NQY * NQ, NP3 = NP * NP * NP;
  __shared__ Tab1d<NP, NQ, NQY> T;
  __shared__ PsiPoly<NP, NQ, NQY> L;
  __shared__ double phi[16 * NPT];  // old then new phi_B at the volume points, then r_B
  __shared__ double ab[16 * NP3];   // a_B, old then new
  __shared__ double GC[128];        // G_new, then C
  __shared__ double ut[24], un[24]; // u~ old and new, [c][B] (read before any write: u_new may be u_old)
  const int tid = threadIdx.x;
  const int64_t enr = blockIdx.x;
  const int64_t e = enriched_cell_index(A.nx, A.ny, A.lower_slot, A.nslots, enr);
  load_tab1d<NP, NQ, NQY>(A.tab, A.minv, T, tid);
  // the Gauss points of both rules follow the tables
  const double* gx = A.tab + tab_layout(NP, NQ, NQY).size;
  const double* gy = gx + NQ;
  const double* po = A.psi_old + enr * A.psi_pts * 4;
  const double* pn = A.psi_new + enr * A.psi_pts * 4;
  for (int q = tid; q < NPT; q += kPrjThreads) {
    const int qx = q % NQ, qy = (q / NQ) % NQY, qz = q / (NQ * NQY);
    const double v[3][2] = {{1.0 - gx[qx], gx[qx]}, {1.0 - gy[qy], gy[qy]}, {1.0 - gx[qz], gx[qz]}};
    const double a = po[q * 4], b = pn[q * 4];
#pragma unroll
    for (int B = 0; B < 8; ++B) {
      const double nb = v[0][B & 1] * v[1][(B >> 1) & 1] * v[2][B >> 2];
      phi[B * NPT + q] = a * nb;
      phi[(8 + B) * NPT + q] = b * nb;
    }
  }
  const int64_t eo = A.ncell * 3 * NP3 + enr * 24;
  if (tid < 24) ut[tid] = A.u_old[eo + tid];
  __syncthreads();
  for (int pr = 0; pr < 8; ++pr) {
    const double* src[2] = {phi + 2 * pr * NPT, phi + (2 * pr + 1) * NPT};
    psi_poly_part<2, NP, NQ, NQY, 1>(src, T, L, tid);
    for (int i = tid; i < 2 * NP3; i += kPrjThreads) ab[2 * pr * NP3 + i] = L.b[i];
    for (int q = tid; q < 2 * NPT; q += kPrjThreads) phi[2 * pr * NPT + q] = L.r[q];
    __syncthreads();
  }
  if (tid < 128) {
    const int j = tid & 7, i = (tid >> 3) & 7, cross = tid >> 6;  // GC[64 cross + 8 i + j]
    const double* ri = phi + (8 + i) * NPT;
    const double* rj = phi + (cross ? j : 8 + j) * NPT;
    double g = 0.0;
    for (int q = 0; q < NPT; ++q) {
      const int qx = q % NQ, qy = (q / NQ) % NQY, qz = q / (NQ * NQY);
      g += T.W[qx] * T.Wy[qy] * T.W[qz] * ri[q] * rj[q];
    }
    GC[tid] = g;
  }
  __syncthreads();
  if (tid == 0) {
    // G_new = C_h C_h^T (Cholesky), then u~_new,c = G_new^{-1} (C u~_old,c)
    double ch[8][8] = {};
    bool ok = A.act_new[enr] != 0;
    for (int j = 0; j < 8 && ok; ++j) {
      double d = GC[j * 8 + j];
      for (int k = 0; k < j; ++k) d -= ch[j][k] * ch[j][k];
      if (!(d > 0.0)) {
        ok = false;
        break;
      }
      ch[j][j] = sqrt(d);
      for (int i = j + 1; i < 8; ++i) {
        double v = GC[i * 8 + j];
        for (int k = 0; k < j; ++k) v -= ch[i][k] * ch[j][k];
        ch[i][j] = v / ch[j][j];
      }
    }
    for (int c = 0; c < 3; ++c) {
      double y[8];
      for (int i = 0; i < 8; ++i) {
        double v = 0.0;
        for (int j = 0; j < 8; ++j) v += GC[64 + i * 8 + j] * ut[c * 8 + j];
        for (int k = 0; k < i; ++k) v -= ch[i][k] * y[k];
        y[i] = ok ? v / ch[i][i] : 0.0;
      }
      for (int i = 7; i >= 0; --i) {
        double v = y[i];
        for (int k = i + 1; k < 8; ++k) v -= ch[k][i] * un[c * 8 + k];
        un[c * 8 + i] = ok ? v / ch[i][i] : 0.0;
      }
    }
  }
  __syncthreads();
  // each entry is read and written by the same thread, so u_new may alias u_old
  const double* ub = A.u_old + e * 3 * NP3;
  double* vb = A.u_new + e * 3 * NP3;
  for (int it = tid; it < 3 * NP3; it += kPrjThreads) {
    const int c = it / NP3, B = it - c * NP3;
    double v = ub[it];
#pragma unroll
    for (int b = 0; b < 8; ++b) v += ut[c * 8 + b] * ab[b * NP3 + B] - un[c * 8 + b] * ab[(8 + b) * NP3 + B];
    vb[it] = v;
  }
  if (tid < 24) A.u_new[eo + tid] = un[tid];
}

// ---------------------------------------------------------------------------
// Inverse velocity mass matrix, x = M^{-1} r (M du/dt = -R(u)).
//
// Regular cell: M = |det J| Kz (x) Ky (x) Kx per component with the cell's
// nq^3 rule, so x = |det J|^{-1} (Kz^{-1} (x) Ky^{-1} (x) Kx^{-1}) r: three
// sweeps through LDS, HBM-bound (16 B per unknown).
// Enriched cell (local basis N_B and psi, rule nq x nqy x nq): with
// K = the polynomial block / |det J|, a = K^{-1} (N, psi)_w and
// s = |det J| (r_psi, r_psi)_w (r_psi = psi - P psi), the Schur complement on
// the enrichment row gives
//   x~ = (r~ - a . r_bar) / s,   x_bar = |det J|^{-1} K^{-1} r_bar - a x~;
// a cell whose enrichment is switched off gets x~ = 0.

struct InvMassArgs {
  int nx, ny, nz, lower_slot, upper_slot, nslots, psi_pts;
  int64_t ncell;
  double ihx, ihz;
  const double* ihy;      // reciprocal cell heights
  const double* tab;
  const double* minv;
  const double* psi;
  const int32_t* act;
  double* apoly;          // [enr][apoly_stride]: a, 1/(r_psi, r_psi)_w (0: enrichment off), (N, psi)_w, (psi, psi)_w
  const double* r;
  double* x;
};

// Per enriched cell: a = K^{-1} (N, psi)_w, 1/(r_psi, r_psi)_w, (N, psi)_w,
// (psi, psi)_w (weights without |det J|).
__host__ __device__ constexpr int apoly_stride(int np3) { return 2 * np3 + 2; }

// The polynomial part of each enriched cell's current psi, cached for the
// inverse mass and the projection step.
template <int NP, int NQ, int NQY>
__global__ __launch_bounds__(kPrjThreads) void psi_poly_kernel(const InvMassArgs A) {
  constexpr int NPT = NQ * NQY * NQ, NP3 = NP * NP * NP;
  __shared__ Tab1d<NP, NQ, NQY> T;
  __shared__ PsiPoly<NP, NQ, NQY> L;
  __shared__ double red[2 * (kPrjThreads / 64)];
  const int tid = threadIdx.x;
  const int64_t enr = blockIdx.x;
  load_tab1d<NP, NQ, NQY>(A.tab, A.minv, T, tid);
  __syncthreads();
  const double* psi[1] = {A.psi + enr * A.psi_pts * 4};
  double* out = A.apoly + enr * apoly_stride(NP3);
  psi_poly_part<1, NP, NQ, NQY>(psi, T, L, tid, out + NP3 + 1);
  double v[2] = {0.0, 0.0};
  for (int q = tid; q < NPT; q += kPrjThreads) {
    const int qx = q % NQ, qy = (q / NQ) % NQY, qz = q / (NQ * NQY);
    const double w = T.W[qx] * T.Wy[qy] * T.W[qz], ps = L.r[q] + L.f[q];  // r = psi - P psi, f = P psi
    v[0] += w * L.r[q] * L.r[q];
    v[1] += w * ps * ps;
  }
  block_sum<2>(v, red, tid);
  for (int B = tid; B < NP3; B += kPrjThreads) out[B] = L.b[B];
  if (tid == 0) {
    out[NP3] = (A.act[enr] && v[0] > 0.0) ? 1.0 / v[0] : 0.0;
    out[2 * NP3 + 1] = v[1];
  }
}

// Degree-1 enrichment weights (Sec. 3.1, eq. enrichment, l = 1): the eight
// enrichment functions phi_B = psi N_B of an enriched cell, N_B its trilinear
// vertex functions (B = bx + 2 (by + 2 bz)).  With a_B = K^{-1} (N, phi_B)_w
// and the residual functions r_B = phi_B - P phi_B, the Schur complement of
// the cell's mass block on its 8 enrichment rows (per component) is |det J| G,
// G_BB' = (r_B, r_B')_w, formed from the pointwise residuals like the l = 0
// (r_psi, r_psi).  Cached per enriched cell: a_0 .. a_7, then G^{-1} (zero
// while the enrichment is switched off).
__host__ __device__ constexpr int apoly_l1_stride(int np3) { return 8 * np3 + 64; }

template <int NP, int NQ, int NQY>
__global__ __launch_bounds__(kPrjThreads) void psi_poly_l1_kernel(const InvMassArgs A) {
  constexpr int NPT = NQ * NQY * NQ, NP3 = NP * NP * NP;
  __shared__ Tab1d<NP, NQ, NQY> T;
  __shared__ PsiPoly<NP, NQ, NQY> L;
  __shared__ double phi[8 * NPT];  // phi_B at the volume points, then r_B
  __shared__ double G[64];
  const int tid = threadIdx.x;
  const int64_t enr = blockIdx.x;
  load_tab1d<NP, NQ, NQY>(A.tab, A.minv, T, tid);
  // the Gauss points of both rules follow the tables
  const double* gx = A.tab + tab_layout(NP, NQ, NQY).size;
  const double* gy = gx + NQ;
  const double* ps = A.psi + enr * A.psi_pts * 4;
  for (int q = tid; q < NPT; q += kPrjThreads) {
    const int qx = q % NQ, qy = (q / NQ) % NQY, qz = q / (NQ * NQY);
    const double v[3][2] = {{1.0 - gx[qx], gx[qx]}, {1.0 - gy[qy], gy[qy]}, {1.0 - gx[qz], gx[qz]}};
    const double p = ps[q * 4];
#pragma unroll
    for (int B = 0; B < 8; ++B) phi[B * NPT + q] = p * (v[0][B & 1] * v[1][(B >> 1) & 1] * v[2][B >> 2]);
  }
  __syncthreads();
  double* out = A.apoly + enr * apoly_l1_stride(NP3);
  for (int pr = 0; pr < 4; ++pr) {
    const double* src[2] = {phi + 2 * pr * NPT, phi + (2 * pr + 1) * NPT};
    psi_poly_part<2, NP, NQ, NQY, 1>(src, T, L, tid);
    for (int i = tid; i < 2 * NP3; i += kPrjThreads) out[2 * pr * NP3 + i] = L.b[i];
    for (int q = tid; q < 2 * NPT; q += kPrjThreads) phi[2 * pr * NPT + q] = L.r[q];
    __syncthreads();
  }
  if (tid < 64) {
    const int B = tid & 7, Bp = tid >> 3;
    double g = 0.0;
    for (int q = 0; q < NPT; ++q) {
      const int qx = q % NQ, qy = (q / NQ) % NQY, qz = q / (NQ * NQY);
      g += T.W[qx] * T.Wy[qy] * T.W[qz] * phi[B * NPT + q] * phi[Bp * NPT + q];
    }
    G[tid] = g;
  }
  __syncthreads();
  if (tid == 0) {
    // G = C C^T (Cholesky), G^{-1} = C^{-T} C^{-1}
    double c[8][8] = {}, ci[8][8] = {};
    bool ok = A.act[enr] != 0;
    for (int j = 0; j < 8 && ok; ++j) {
      double d = G[j * 8 + j];
      for (int k = 0; k < j; ++k) d -= c[j][k] * c[j][k];
      if (!(d > 0.0)) {
        ok = false;
        break;
      }
      c[j][j] = sqrt(d);
      for (int i = j + 1; i < 8; ++i) {
        double v = G[i * 8 + j];
        for (int k = 0; k < j; ++k) v -= c[i][k] * c[j][k];
        c[i][j] = v / c[j][j];
      }
    }
    if (ok)
      for (int j = 0; j < 8; ++j) {  // columns of C^{-1} by forward substitution
        for (int i = 0; i < 8; ++i) {
          double v = i == j ? 1.0 : 0.0;
          for (int k = 0; k < i; ++k) v -= c[i][k] * ci[k][j];
          ci[i][j] = v / c[i][i];
        }
      }
    for (int i = 0; i < 8; ++i)
      for (int j = 0; j < 8; ++j) {
        double v = 0.0;
        if (ok)
          for (int k = 0; k < 8; ++k) v += ci[k][i] * ci[k][j];
        out[8 * NP3 + i * 8 + j] = v;
      }
  }
}

constexpr int kImThreads = 64;

// x = M^{-1} r, one wavefront per cell.  ENR = false: regular cells, block
// b = ex + nx (ly + nlayers ez) with ey = layer_lo + ly; ENR = true: block b
// = enriched index.  The cell sits in LDS once and each 1-D sweep runs in
// place, one line per lane (a lane reads its whole line into registers
// before writing it back), with the inverse 1-D mass matrix in registers.
// Enriched cells use the wall-normal rule's matrix along y and the cached
// polynomial part of psi:
//   x~_c = (r~_c - a . r_bar_c) / (|det J| (r_psi, r_psi)),
//   x_bar_c = |det J|^{-1} K^{-1} r_bar_c - a x~_c.
template <int NP, bool ENR, int LE = 1>
__global__ __launch_bounds__(kImThreads) void invmass_kernel(const InvMassArgs A, int layer_lo, int nlayers) {
  constexpr int NP2 = NP * NP, NP3 = NP2 * NP;
  __shared__ double u[3 * NP3];
  __shared__ double sa[ENR ? LE * NP3 : 1];
  __shared__ double sxt[3 * LE];  // l = 1: the enrichment unknowns [c][B]
  __shared__ double sd[3 * LE];   // l = 1: r~ - A r_bar
  const int tid = threadIdx.x;
  const int64_t b = blockIdx.x;
  int64_t e;
  int ey;
  if (ENR) {
    e = enriched_cell_index(A.nx, A.ny, A.lower_slot, A.nslots, b);
    ey = (int)((e / A.nx) % A.ny);
  } else {
    const int ex = (int)(b % A.nx);
    const int64_t t0 = b / A.nx;
    ey = layer_lo + (int)(t0 % nlayers);
    e = ex + (int64_t)A.nx * (ey + (int64_t)A.ny * (t0 / nlayers));
  }
  const double* re = A.r + e * 3 * NP3;
  for (int i = tid; i < 3 * NP3; i += kImThreads) u[i] = re[i];
  double m[NP2];
#pragma unroll
  for (int i = 0; i < NP2; ++i) m[i] = A.minv[i];
  const double idet = A.ihx * A.ihy[ey] * A.ihz;
  double xt0 = 0.0, xt1 = 0.0, xt2 = 0.0;
  if constexpr (ENR && LE == 8) {
    // degree-1 weights: x~_c = |det J|^{-1} G^{-1} (r~_c - A r_bar_c), A = [a_B]
    const double* ap = A.apoly + b * apoly_l1_stride(NP3);
    for (int i = tid; i < 8 * NP3; i += kImThreads) sa[i] = ap[i];
    __syncthreads();
    double d[24];
#pragma unroll
    for (int i = 0; i < 24; ++i) d[i] = 0.0;
    for (int i = tid; i < NP3; i += kImThreads) {
#pragma unroll
      for (int B = 0; B < 8; ++B) {
        const double ab = sa[B * NP3 + i];
        d[B] += ab * u[i];
        d[8 + B] += ab * u[NP3 + i];
        d[16 + B] += ab * u[2 * NP3 + i];
      }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
#pragma unroll
      for (int i = 0; i < 24; ++i) d[i] += __shfl_xor(d[i], off, 64);
    const int64_t eo = A.ncell * 3 * NP3 + b * 24;
    if (tid == 0)
#pragma unroll
      for (int i = 0; i < 24; ++i) sd[i] = A.r[eo + i] - d[i];  // r~_c - A r_bar_c
    __syncthreads();
    if (tid < 24) {
      const int c = tid >> 3, B = tid & 7;
      double x = 0.0;
#pragma unroll
      for (int Bp = 0; Bp < 8; ++Bp) x += ap[8 * NP3 + B * 8 + Bp] * sd[c * 8 + Bp];
      sxt[tid] = x * idet;
    }
    __syncthreads();  // every lane has read u and r~ before anything is overwritten
    if (tid < 24) A.x[eo + tid] = sxt[tid];
  } else if (ENR) {
    const double* ap = A.apoly + b * apoly_stride(NP3);
    for (int i = tid; i < NP3; i += kImThreads) sa[i] = ap[i];
    __syncthreads();
    double d0 = 0.0, d1 = 0.0, d2 = 0.0;
    for (int B = tid; B < NP3; B += kImThreads) {
      const double ab = sa[B];
      d0 += ab * u[B];
      d1 += ab * u[NP3 + B];
      d2 += ab * u[2 * NP3 + B];
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      d0 += __shfl_xor(d0, off, 64);
      d1 += __shfl_xor(d1, off, 64);
      d2 += __shfl_xor(d2, off, 64);
    }
    const double is = ap[NP3] * idet;
    const int64_t eo = A.ncell * 3 * NP3 + b * 3;
    xt0 = (A.r[eo + 0] - d0) * is;
    xt1 = (A.r[eo + 1] - d1) * is;
    xt2 = (A.r[eo + 2] - d2) * is;
    __syncthreads();  // every lane has read u and r~ before anything is overwritten
    if (tid == 0) {
      A.x[eo + 0] = xt0;
      A.x[eo + 1] = xt1;
      A.x[eo + 2] = xt2;
    }
  } else {
    __syncthreads();
  }
  // lines along x (c, j, k): base c NP3 + NP (j + NP k), stride 1
  for (int L = tid; L < 3 * NP2; L += kImThreads) {
    double* p = u + (L / NP2) * NP3 + (L % NP2) * NP;
    double x[NP];
#pragma unroll
    for (int l = 0; l < NP; ++l) x[l] = p[l];
#pragma unroll
    for (int o = 0; o < NP; ++o) {
      double s = 0.0;
#pragma unroll
      for (int l = 0; l < NP; ++l) s += m[o * NP + l] * x[l];
      p[o] = s;
    }
  }
  __syncthreads();
  if (ENR) {
#pragma unroll
    for (int i = 0; i < NP2; ++i) m[i] = A.minv[NP2 + i];
  }
  // lines along y (c, i, k): base c NP3 + i + NP2 k, stride NP
  for (int L = tid; L < 3 * NP2; L += kImThreads) {
    const int ik = L % NP2;
    double* p = u + (L / NP2) * NP3 + (ik % NP) + NP2 * (ik / NP);
    double x[NP];
#pragma unroll
    for (int l = 0; l < NP; ++l) x[l] = p[l * NP];
#pragma unroll
    for (int o = 0; o < NP; ++o) {
      double s = 0.0;
#pragma unroll
      for (int l = 0; l < NP; ++l) s += m[o * NP + l] * x[l];
      p[o * NP] = s;
    }
  }
  __syncthreads();
  if (ENR) {
#pragma unroll
    for (int i = 0; i < NP2; ++i) m[i] = A.minv[i];
  }
  // lines along z (c, i, j): base c NP3 + i + NP j, stride NP2, straight to memory
  double* xe = A.x + e * 3 * NP3;
  for (int L = tid; L < 3 * NP2; L += kImThreads) {
    const int c = L / NP2, b0 = L % NP2;
    const double* p = u + c * NP3 + b0;
    const double xc = c == 0 ? xt0 : (c == 1 ? xt1 : xt2);
    double x[NP];
#pragma unroll
    for (int l = 0; l < NP; ++l) x[l] = p[l * NP2];
#pragma unroll
    for (int o = 0; o < NP; ++o) {
      double s = 0.0;
#pragma unroll
      for (int l = 0; l < NP; ++l) s += m[o * NP + l] * x[l];
      s *= idet;
      if constexpr (ENR && LE == 1) s -= sa[b0 + o * NP2] * xc;
      if constexpr (ENR && LE == 8) {
#pragma unroll
        for (int B = 0; B < 8; ++B) s -= sa[B * NP3 + b0 + o * NP2] * sxt[c * 8 + B];
      }
      xe[c * NP3 + b0 + o * NP2] = s;
    }
  }
}

// ---------------------------------------------------------------------------
template <int NP, int NQ>
using MSt = ct::MatS<NP, NQ>;
template <int NP, int NQ>
using MDt = ct::MatSd<NP, NQ>;

// Element-wise projection step (Sec. 4.2, eq. projectionspat),
//   (M_e + D_e) x = M_e u_hat - scale g,   D_e(v, w) = (div v, tau_D,e div w)_e,
// solved directly in enriched cells.  The
// polynomial block of an enriched cell is the block of a cell without
// enrichment of the same height (both Gauss rules integrate the polynomial
// products exactly), P = |J| (Mh + tau Dh), solved with the layer's spectral
// tables.  The enrichment unknowns are taken in the basis r e_d, r = psi - P psi
// (P psi = sum_B a_B N_B, the L2 projection of the cached polynomial part),
// which is mass-orthogonal to the polynomials: u = sum x'_B N_B + x_e r with
// x_p = x'_p - a x_e.  In that basis (all entries divided by |J|, weights
// without |J|)
//   C'_d[c][B] = tau (d N_B / d x_c, d r / d x_d)_w,
//   E'_cd = delta_cd (r, r)_w + tau (d r / d x_c, d r / d x_d)_w,
//   b'_e,d = (r, r)_w u_e,d - (s/|J|) (g_e,d - sum_B a_B g_p[d][B]),
// so the mass part of the Schur complement S' = E' - C'^T P^{-1} C' is the
// exact (r, r) and nothing cancels as tau -> 0 (as for the inverse mass).
// The four right-hand sides b_p, C'_0, C'_1, C'_2 of a cell take the first
// spectral product together; every C'^T P^{-1} (.) is then a weighted dot
// product of its outputs, sum_r y_j[r] y_k[r] / (1 + tau lambda_r); and by
// linearity only x'_p = P^{-1} (b_p - C' x_e) takes the second product.  Four
// cells per workgroup, one wavefront per cell in the dense products.  A cell
// whose enrichment is off has x_e = 0 and x_p = P^{-1} b_p.
struct BorderArgs {
  InvMassArgs im;
  const double* mats;   // K^{-1}, C^T, C^{-T}
  const double* slots;  // per layer slot: (L Z)^T and L^{-T} Z tables, lambda
  const int32_t* map;
  const double* tau_d;
  const double* u_hat;
  const double* g;
  double scale;
  double* x;
  const double* coup;   // [enr][coup_stride]: coupling columns and (grad r, grad r)_w
  int tiles;            // tiles of four cells per enriched layer
  int64_t ncol;         // cells per layer
};

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Per enriched cell, the psi-dependent parts of the bordered projection
// step (they change only with psi; cached like the polynomial part):
//   t'_d[c][B] = (d N_B / d x_c, d r / d x_d)_w  (3 x 3 NP^3, d-major), then
//   (d r / d x_c, d r / d x_d)_w  for cd = 00 01 02 11 12 22,
// with grad r = grad psi - grad P psi at the enriched volume points (weights
// without |J|, physical derivatives).
__host__ __device__ constexpr int coup_stride(int np3) { return 9 * np3 + 6; }

template <int NP, int NQ, int NQY>
__global__ __launch_bounds__(kSpecThreads) void coupling_kernel(const InvMassArgs A, double* coup) {
  constexpr int NP3 = NP * NP * NP, NPT = NQ * NQY * NQ;
  constexpr auto& tq = ct::tab<NP, NQ>;
  constexpr auto& ty = ct::tab<NP, NQY>;
  __shared__ double W0[9 * NPT], W1[9 * NPT], OUT[9 * NP3];
  __shared__ double Av[NP3];
  __shared__ double red[6 * (kSpecThreads / 64)];
  const int tid = threadIdx.x;
  const int64_t b = blockIdx.x;
  const int64_t e = enriched_cell_index(A.nx, A.ny, A.lower_slot, A.nslots, b);
  const int ey = (int)((e / A.nx) % A.ny);
  const double h[3] = {1.0 / A.ihx, 1.0 / A.ihy[ey], 1.0 / A.ihz};
  const double* ps = A.psi + b * A.psi_pts * 4;
  for (int B = tid; B < NP3; B += kSpecThreads) Av[B] = A.apoly[b * apoly_stride(NP3) + B];
  __syncthreads();
  // reference gradient of P psi at the points: W0[d][q]
  sweep_c<0, NP, NP, NP, NQ, false, false, MDt<NP, NQ>>(Av, NP3, W1, NPT, 1.0, 1, 0);
  sweep_c<0, NP, NP, NP, NQ, false, false, MSt<NP, NQ>>(Av, NP3, W1 + NPT, NPT, 1.0, 1, 64);
  __syncthreads();
  sweep_c<1, NQ, NP, NP, NQY, false, false, MSt<NP, NQY>>(W1, NPT, W1 + 2 * NPT, NPT, 1.0, 1, 0);
  sweep_c<1, NQ, NP, NP, NQY, false, false, MDt<NP, NQY>>(W1 + NPT, NPT, W1 + 3 * NPT, NPT, 1.0, 1, 64);
  sweep_c<1, NQ, NP, NP, NQY, false, false, MSt<NP, NQY>>(W1 + NPT, NPT, W1 + 4 * NPT, NPT, 1.0, 1, 128);
  __syncthreads();
  sweep_c<2, NQ, NQY, NP, NQ, false, false, MSt<NP, NQ>>(W1 + 2 * NPT, NPT, W0, NPT, 1.0, 2, 0);
  sweep_c<2, NQ, NQY, NP, NQ, false, false, MDt<NP, NQ>>(W1 + 4 * NPT, NPT, W0 + 2 * NPT, NPT, 1.0, 1, 128);
  __syncthreads();
  double e6[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (int q = tid; q < NPT; q += kSpecThreads) {
    const int qx = q % NQ, qy = (q / NQ) % NQY, qz = q / (NQ * NQY);
    const double w = tq.w[qx] * ty.w[qy] * tq.w[qz];
    double gr[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) gr[d] = ps[q * 4 + 1 + d] - W0[d * NPT + q] / h[d];
    e6[0] += w * gr[0] * gr[0];
    e6[1] += w * gr[0] * gr[1];
    e6[2] += w * gr[0] * gr[2];
    e6[3] += w * gr[1] * gr[1];
    e6[4] += w * gr[1] * gr[2];
    e6[5] += w * gr[2] * gr[2];
#pragma unroll
    for (int cc = 0; cc < 3; ++cc)
#pragma unroll
      for (int d = 0; d < 3; ++d) W1[(cc * 3 + d) * NPT + q] = w * gr[d] / h[cc];  // [component][d][q]
  }
  block_sum<6>(e6, red, tid);  // (its barriers also publish W1)
  double* out = coup + b * coup_stride(NP3);
  if (tid < 6) out[9 * NP3 + tid] = e6[tid];
  sweep_c<0, NQ, NQY, NQ, NP, true, false, MDt<NP, NQ>>(W1, NPT, W0, NPT, 1.0, 3, 0);
  sweep_c<0, NQ, NQY, NQ, NP, true, false, MSt<NP, NQ>>(W1 + 3 * NPT, NPT, W0 + 3 * NPT, NPT, 1.0, 6, 64);
  __syncthreads();
  sweep_c<1, NP, NQY, NQ, NP, true, false, MSt<NP, NQY>>(W0, NPT, W1, NPT, 1.0, 3, 0);
  sweep_c<1, NP, NQY, NQ, NP, true, false, MDt<NP, NQY>>(W0 + 3 * NPT, NPT, W1 + 3 * NPT, NPT, 1.0, 3, 64);
  sweep_c<1, NP, NQY, NQ, NP, true, false, MSt<NP, NQY>>(W0 + 6 * NPT, NPT, W1 + 6 * NPT, NPT, 1.0, 3, 128);
  __syncthreads();
  sweep_c<2, NP, NP, NQ, NP, true, false, MSt<NP, NQ>>(W1, NPT, OUT, NP3, 1.0, 6, 0);
  sweep_c<2, NP, NP, NQ, NP, true, false, MDt<NP, NQ>>(W1 + 6 * NPT, NPT, OUT + 6 * NP3, NP3, 1.0, 3, 128);
  __syncthreads();
  for (int it = tid; it < 9 * NP3; it += kSpecThreads) {
    const int d = it / (3 * NP3), k = it - d * 3 * NP3, cc = k / NP3, B = k - cc * NP3;
    out[it] = OUT[(cc * 3 + d) * NP3 + B];
  }
}

template <int NP, int NQ, int NQY>
__global__ __launch_bounds__(kSpecThreads) void bordered_step_kernel(const BorderArgs S) {
  constexpr int NP2 = NP * NP, NP3 = NP2 * NP, N = 3 * NP3, NC = 16, LD = NC + 2;
  __shared__ double T[N * LD];
  __shared__ double Mt[3 * NP2];
  __shared__ double XE[4][3];
  const InvMassArgs& A = S.im;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int slot = blockIdx.x / S.tiles;
  const int64_t j0 = (int64_t)(blockIdx.x % S.tiles) * 4;
  const int nc = S.ncol - j0 < 4 ? (int)(S.ncol - j0) : 4;
  const int ey = slot == A.lower_slot ? 0 : A.ny - 1;
  const double h[3] = {1.0 / A.ihx, 1.0 / A.ihy[ey], 1.0 / A.ihz};
  const double detJ = h[0] * h[1] * h[2], f = S.scale / detJ;
  // cell c of the tile: enriched index and cell index
  auto enr_of = [&](int c) -> int64_t {
    const int64_t j = j0 + c;
    return j % A.nx + (int64_t)A.nx * (slot + (int64_t)A.nslots * (j / A.nx));
  };
  auto cell_of = [&](int c) -> int64_t {
    const int64_t j = j0 + c;
    return j % A.nx + (int64_t)A.nx * (ey + (int64_t)A.ny * (j / A.nx));
  };
  for (int i = tid; i < 3 * NP2; i += kSpecThreads) Mt[i] = S.mats[i];
  // columns: -f g_p, then tau t'_d (zero in padding cells)
  for (int it = tid; it < 4 * 4 * N; it += kSpecThreads) {
    const int c = it / (4 * N), r = it - c * 4 * N, col = r / N, k = r - col * N;
    double v = 0.0;
    if (c < nc) {
      if (col == 0)
        v = -f * S.g[cell_of(c) * N + k];
      else
        v = S.tau_d[cell_of(c)] * S.coup[enr_of(c) * coup_stride(NP3) + (col - 1) * N + k];
    }
    T[k * LD + 4 * c + col] = v;
  }
  __syncthreads();
  // Mh^{-1} on all columns; column 0 becomes Mh^{-1} b_p = u_p + a u_e - f Mh^{-1} g_p
  tile_sweep<NP, NC, 0>(T, Mt, tid);
  __syncthreads();
  tile_sweep<NP, NC, 1>(T, Mt, tid);
  __syncthreads();
  tile_sweep<NP, NC, 2>(T, Mt, tid);
  __syncthreads();
  for (int it = tid; it < 4 * N; it += kSpecThreads) {
    const int c = it / N, k = it - c * N, cc = k / NP3, B = k - cc * NP3;
    if (c >= nc) continue;
    const int64_t b = enr_of(c);
    const double a = A.apoly[b * apoly_stride(NP3) + B];
    T[k * LD + 4 * c] += S.u_hat[cell_of(c) * N + k] + a * S.u_hat[A.ncell * N + 3 * b + cc];
  }
  __syncthreads();
  // per-cell scalars: wavefront wv <-> cell wv
  __shared__ double TAU[4], Gp[2][4][9];
  const bool valid = wv < nc;
  const int64_t b = valid ? enr_of(wv) : 0;
  const int64_t e = valid ? cell_of(wv) : 0;
  const double tau = valid ? S.tau_d[e] : 0.0;
  const double* ap = A.apoly + b * apoly_stride(NP3);
  const bool on = valid && ap[NP3] != 0.0;
  double ag[3] = {0.0, 0.0, 0.0};  // sum_B a_B g_p[d][B]
  if (on) {
    const double* gp = S.g + e * N;
    for (int B = lane; B < NP3; B += 64) {
      const double aB = ap[B];
      ag[0] += aB * gp[B];
      ag[1] += aB * gp[NP3 + B];
      ag[2] += aB * gp[2 * NP3 + B];
    }
  }
#pragma unroll
  for (int i = 0; i < 3; ++i) ag[i] = wave_sum(ag[i]);
  if (lane == 0) TAU[wv] = tau;
  const int32_t lslot = S.map[ey];
  const double* Zs = S.slots + (size_t)lslot * (2 * (size_t)N * N + N);
  const double* lam = Zs + 2 * (size_t)N * N;
  __syncthreads();
  // dense products split 2 x 2: wavefront (rw, cw) takes row chunks rw + 2 i
  // and the columns of cells 2 cw, 2 cw + 1
  constexpr int WR = 2, CPW = 8, RPW = ((N + 63) / 64 + WR - 1) / WR;
  const int rw = wv % WR, cw = wv / WR;
  double acc[RPW][CPW];
  tile_gemm_split<N, LD, WR, RPW, CPW>(T, Zs, acc, lane, wv);
  // weighted dot products G_jk = sum_r y_j[r] y_k[r] / (1 + tau lambda_r), partial over this row half
  double sr[RPW][2];
  double Gl[2][9];
#pragma unroll
  for (int m = 0; m < 2; ++m)
#pragma unroll
    for (int k = 0; k < 9; ++k) Gl[m][k] = 0.0;
#pragma unroll
  for (int i = 0; i < RPW; ++i) {
    const int r = 64 * (rw + WR * i) + lane;
    const double lr = r < N ? lam[r] : 0.0;
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      const double w = r < N ? 1.0 / (1.0 + TAU[2 * cw + m] * lr) : 0.0;
      sr[i][m] = w;
      const double y0 = acc[i][4 * m], y1 = acc[i][4 * m + 1], y2 = acc[i][4 * m + 2], y3 = acc[i][4 * m + 3];
      Gl[m][0] += w * y1 * y0;  // 10 20 30 11 12 13 22 23 33
      Gl[m][1] += w * y2 * y0;
      Gl[m][2] += w * y3 * y0;
      Gl[m][3] += w * y1 * y1;
      Gl[m][4] += w * y1 * y2;
      Gl[m][5] += w * y1 * y3;
      Gl[m][6] += w * y2 * y2;
      Gl[m][7] += w * y2 * y3;
      Gl[m][8] += w * y3 * y3;
    }
  }
#pragma unroll
  for (int m = 0; m < 2; ++m)
#pragma unroll
    for (int k = 0; k < 9; ++k) Gl[m][k] = wave_sum(Gl[m][k]);
  if (lane == 0)
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
      for (int k = 0; k < 9; ++k) Gp[rw][2 * cw + m][k] = Gl[m][k];
  __syncthreads();  // every wavefront is done reading T; partial sums published
  double G[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) G[k] = Gp[0][wv][k] + Gp[1][wv][k];
  double xe[3] = {0.0, 0.0, 0.0};
  if (on) {
    const double rr = 1.0 / ap[NP3];
    const double* ue = S.u_hat + A.ncell * N + 3 * b;
    const double* ge = S.g + A.ncell * N + 3 * b;
    const double* E = S.coup + b * coup_stride(NP3) + 9 * NP3;
    // S' = E' - C'^T P^{-1} C' and rhs = b'_e - C'^T P^{-1} b_p (all divided by |J|)
    const double s00 = rr + tau * E[0] - G[3], s01 = tau * E[1] - G[4], s02 = tau * E[2] - G[5];
    const double s11 = rr + tau * E[3] - G[6], s12 = tau * E[4] - G[7], s22 = rr + tau * E[5] - G[8];
    const double r0 = rr * ue[0] - f * (ge[0] - ag[0]) - G[0];
    const double r1 = rr * ue[1] - f * (ge[1] - ag[1]) - G[1];
    const double r2 = rr * ue[2] - f * (ge[2] - ag[2]) - G[2];
    // symmetric 3 x 3 solve by cofactors
    const double c00 = s11 * s22 - s12 * s12, c01 = s02 * s12 - s01 * s22, c02 = s01 * s12 - s02 * s11;
    const double c11 = s00 * s22 - s02 * s02, c12 = s01 * s02 - s00 * s12, c22 = s00 * s11 - s01 * s01;
    const double idet = 1.0 / (s00 * c00 + s01 * c01 + s02 * c02);
    xe[0] = (c00 * r0 + c01 * r1 + c02 * r2) * idet;
    xe[1] = (c01 * r0 + c11 * r1 + c12 * r2) * idet;
    xe[2] = (c02 * r0 + c12 * r1 + c22 * r2) * idet;
  }
  if (lane == 0)
#pragma unroll
    for (int d = 0; d < 3; ++d) XE[wv][d] = xe[d];
  __syncthreads();  // XE published
#pragma unroll
  for (int i = 0; i < RPW; ++i) {
    const int r = 64 * (rw + WR * i) + lane;
    if (r < N)
#pragma unroll
      for (int m = 0; m < 2; ++m) {
        const int cl = 2 * cw + m;
        T[r * LD + 4 * cl] = (acc[i][4 * m] - XE[cl][0] * acc[i][4 * m + 1] - XE[cl][1] * acc[i][4 * m + 2] -
                              XE[cl][2] * acc[i][4 * m + 3]) * sr[i][m];
      }
  }
  __syncthreads();
  tile_gemm_split<N, LD, WR, RPW, CPW>(T, Zs + (size_t)N * N, acc, lane, wv);
  __syncthreads();
#pragma unroll
  for (int i = 0; i < RPW; ++i) {
    const int r = 64 * (rw + WR * i) + lane;
    if (r < N)
#pragma unroll
      for (int m = 0; m < 2; ++m) T[r * LD + 4 * (2 * cw + m)] = acc[i][4 * m];
  }
  __syncthreads();
  // back to the psi basis: x_p = x'_p - a x_e
  for (int it = tid; it < 4 * N; it += kSpecThreads) {
    const int c = it / N, k = it - c * N, cc = k / NP3, B = k - cc * NP3;
    if (c < nc)
      S.x[cell_of(c) * N + k] = T[k * LD + 4 * c] - A.apoly[enr_of(c) * apoly_stride(NP3) + B] * XE[c][cc];
  }
  if (valid && lane < 3) S.x[A.ncell * N + 3 * b + lane] = XE[wv][lane];
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
    if (m->nle == 8)                                                                                \
      hipLaunchKernelGGL((project_l1_kernel<p, q, w>), dim3((unsigned)m->nenr), dim3(kPrjThreads), 0, s, A); \
    else                                                                                            \
      hipLaunchKernelGGL((project_kernel<p, q, w>), dim3((unsigned)m->nenr), dim3(kPrjThreads), 0, s, A); \
    return check_hip(hipGetLastError(), "projection kernel launch");                                \
  }
  DG_PRJ_COMBOS(X)
#undef X
  return set_error(DG_ERR_UNSUPPORTED, "projection: (k_u+1, nq_u, nq_wn) combination not compiled");
}

namespace {

InvMassArgs invmass_args(const dg_mesh* m, const double* r, double* x) {
  InvMassArgs A;
  A.nx = m->P.nx;
  A.ny = m->P.ny;
  A.nz = m->P.nz;
  A.lower_slot = m->lower_slot;
  A.upper_slot = m->upper_slot;
  A.nslots = m->n_enr_layers;
  A.psi_pts = m->psi_pts;
  A.ncell = m->ncell;
  A.ihx = 1.0 / m->hx;
  A.ihz = 1.0 / m->hz;
  A.ihy = m->hy + m->P.ny;
  A.tab = m->tab_u;
  A.minv = m->minv;
  A.psi = m->psi;
  A.act = m->act;
  A.apoly = m->apoly;
  A.r = r;
  A.x = x;
  return A;
}

// Fill the cache of the enriched cells' polynomial parts of psi if the current
// psi table has changed since it was last filled.
int ensure_psi_poly(const dg_mesh* m, const InvMassArgs& A, hipStream_t s) {
  if (m->nenr > 0 && !m->apoly_ok) {
    bool launched = false;
#define X(p, q, w)                                                                                        \
    if (!launched && m->np_u == p && m->P.nq_u == q && m->P.nq_wn == w) {                                 \
      if (m->nle == 8)                                                                                    \
        hipLaunchKernelGGL((psi_poly_l1_kernel<p, q, w>), dim3((unsigned)m->nenr), dim3(kPrjThreads), 0, s, A); \
      else                                                                                                \
        hipLaunchKernelGGL((psi_poly_kernel<p, q, w>), dim3((unsigned)m->nenr), dim3(kPrjThreads), 0, s, A); \
      const int rc = check_hip(hipGetLastError(), "psi polynomial part kernel launch");                   \
      if (rc) return rc;                                                                                  \
      launched = true;                                                                                    \
    }
    DG_PRJ_COMBOS(X)
#undef X
    if (!launched) return set_error(DG_ERR_UNSUPPORTED, "(k_u+1, nq_u, nq_wn) combination not compiled");
    m->apoly_ok = 1;
  }
  return DG_OK;
}

}  // namespace

int launch_inverse_mass(const dg_mesh* m, const double* r, double* x, hipStream_t s) {
  if (m->curved) return launch_inverse_mass_curved(m, r, x, s);
  const InvMassArgs A = invmass_args(m, r, x);
  const int rc0 = ensure_psi_poly(m, A, s);
  if (rc0) return rc0;
  // regular layers: all but the enriched wall-adjacent ones
  const int lo = (m->P.fully_periodic || m->lower_slot < 0) ? 0 : 1;
  const int hi = (m->P.fully_periodic || m->upper_slot < 0) ? m->P.ny - 1 : m->P.ny - 2;
  const int nl = hi - lo + 1;
  const int64_t nreg = nl > 0 ? (int64_t)m->P.nx * nl * m->P.nz : 0;
#define X(p)                                                                                                 \
  if (m->np_u == p) {                                                                                        \
    if (nreg > 0) {                                                                                          \
      hipLaunchKernelGGL((invmass_kernel<p, false>), dim3((unsigned)nreg), dim3(kImThreads), 0, s, A, lo, nl); \
      const int rc = check_hip(hipGetLastError(), "inverse mass kernel launch");                             \
      if (rc) return rc;                                                                                     \
    }                                                                                                        \
    if (m->nenr > 0 && m->nle == 8)                                                                          \
      hipLaunchKernelGGL((invmass_kernel<p, true, 8>), dim3((unsigned)m->nenr), dim3(kImThreads), 0, s, A, 0, 0); \
    else if (m->nenr > 0)                                                                                    \
      hipLaunchKernelGGL((invmass_kernel<p, true>), dim3((unsigned)m->nenr), dim3(kImThreads), 0, s, A, 0, 0); \
    return check_hip(hipGetLastError(), "inverse mass kernel launch");                                       \
  }
  X(3) X(4) X(5) X(6)
#undef X
  return set_error(DG_ERR_UNSUPPORTED, "inverse mass: degree not compiled");
}


int launch_projection_step(const dg_mesh* m, const double* tau_d, const double* u_hat, const double* g, double scale,
                           double* x, hipStream_t s) {
  if (m->P.omit_step_tables)
    return set_error(DG_ERR_UNSUPPORTED, "the mesh was set up without projection-step tables (omit_step_tables)");
  int rc = ensure_spectral_tables(m, s);
  // cells without enrichment: direct solve per layer
  if (!rc) rc = launch_spectral_step(m, tau_d, u_hat, g, scale, x, s);
  if (rc || m->nenr == 0) return rc;
  const InvMassArgs IA = invmass_args(m, nullptr, nullptr);
  rc = ensure_psi_poly(m, IA, s);
  if (rc) return rc;
  if (!m->coup_ok) {
    bool launched = false;
#define X(p, q, w)                                                                                               \
    if (!launched && m->np_u == p && m->P.nq_u == q && m->P.nq_wn == w) {                                        \
      hipLaunchKernelGGL((coupling_kernel<p, q, w>), dim3((unsigned)m->nenr), dim3(kSpecThreads), 0, s, IA,     \
                         m->coup);                                                                               \
      launched = true;                                                                                           \
    }
    DG_PRJ_COMBOS(X)
#undef X
    if (!launched) return set_error(DG_ERR_UNSUPPORTED, "projection step: (k_u+1, nq_u, nq_wn) combination not compiled");
    rc = check_hip(hipGetLastError(), "projection step coupling kernel launch");
    if (rc) return rc;
    m->coup_ok = 1;
  }
  BorderArgs B;
  B.coup = m->coup;
  B.im = IA;
  spectral_pointers(m, &B.mats, &B.slots, &B.map);
  B.tau_d = tau_d;
  B.u_hat = u_hat;
  B.g = g;
  B.scale = scale;
  B.x = x;
  B.ncol = (int64_t)m->P.nx * m->P.nz;
  const int64_t tiles = (B.ncol + 3) / 4;
  if (tiles * m->n_enr_layers > INT32_MAX / 2) return set_error(DG_ERR_ARG, "projection step: mesh too large");
  B.tiles = (int)tiles;
  const int grid = (int)(tiles * m->n_enr_layers);
#define X(p, q, w)                                                                                       \
  if (m->np_u == p && m->P.nq_u == q && m->P.nq_wn == w) {                                               \
    hipLaunchKernelGGL((bordered_step_kernel<p, q, w>), dim3((unsigned)grid), dim3(kSpecThreads), 0, s, B); \
    return check_hip(hipGetLastError(), "projection step kernel launch");                                \
  }
  DG_PRJ_COMBOS(X)
#undef X
  return set_error(DG_ERR_UNSUPPORTED, "projection step: (k_u+1, nq_u, nq_wn) combination not compiled");
}

}  // namespace dgwm
