// Enriched DG velocity residual (arXiv 1705.08813, Sec. 3.1 and 4.2):
// local Lax-Friedrichs convective term + interior-penalty viscous term on the
// space u = u_bar + psi u~ (l = 0 enrichment in the wall-adjacent layer).
//
// One workgroup per cell.  The cell's nodal values are staged in LDS; values
// and gradients at the Gauss points come from sum-factorized sweeps (basis
// interpolation, then collocation derivatives through the Gauss points); the
// pointwise flux is integrated back with the transposed sweeps.  Faces are
// handled element by element: each cell evaluates its own and its
// neighbour's traces on each of its six faces and integrates the numerical
// flux against its own test functions, so every output has one writer and no
// atomics are needed.  Enriched cells run a separate instantiation whose
// wall-normal rule has NQY points and which reads the precomputed psi and
// grad psi tables.
#include "kern_common.h"

namespace dgwm {

namespace {

template <typename T, int NP, int NQ, int NQY>
struct VelShape {
  static constexpr int NP2 = NP * NP, NP3 = NP * NP * NP;
  static constexpr int NPTS = NQ * NQY * NQ;
  static constexpr int FMAX = (NQ * NQY > NQ * NQ) ? NQ * NQY : NQ * NQ;
  static constexpr int LAY = 2 * 3 * 2 * NP2;   // [side][c][value|normal derivative][NP2]
  static constexpr int TR = 2 * 3 * 4 * FMAX;   // [side][c][val|d_t1|d_t2|d_n][FMAX]
  static constexpr int FL = 12 * FMAX;          // [fv c | Fg c k][FMAX]
  static constexpr int FACE = LAY + TR + FL;
  static constexpr int VOL = 12 * NPTS;
  static constexpr int BIG = VOL > FACE ? VOL : FACE;
};

// Processes face (D, S) of the current cell.  T1 < T2 are the tangential
// directions.  Adds the integrated flux to s_r and (enriched cells) to rt.
template <typename T, int NP, int NQ, int NQY, bool ENR, int D, int S>
__device__ __forceinline__ void vel_face(const MeshDev& M, const T* __restrict__ u, const T* s_u, T* s_r,
                                         T* s_big, const T* s_ut, int ex, int ey, int ez, int64_t enr, T hx,
                                         T hy, T hz, T rt[3]) {
  using Sh = VelShape<T, NP, NQ, NQY>;
  constexpr TabLayout L = tab_layout(NP, NQ, NQY);
  constexpr int T1 = D == 0 ? 1 : 0;
  constexpr int T2 = D == 2 ? 1 : 2;
  constexpr int Q1 = T1 == 1 ? NQY : NQ;
  constexpr int Q2 = T2 == 1 ? NQY : NQ;
  constexpr int FP = Q1 * Q2;
  constexpr int NP2 = Sh::NP2, NP3 = Sh::NP3;
  const int tid = threadIdx.x, nt = blockDim.x;
  const double* tab = M.tab;
  const double* Sx = tab + L.S;
  const double* Sdx = tab + L.Sd;
  const double* Sy = ENR ? tab + L.Sy : tab + L.S;
  const double* Sdy = ENR ? tab + L.Sdy : tab + L.Sd;
  const double* St1 = T1 == 1 ? Sy : Sx;
  const double* Sdt1 = T1 == 1 ? Sdy : Sdx;
  const double* St2 = T2 == 1 ? Sy : Sx;
  const double* Sdt2 = T2 == 1 ? Sdy : Sdx;
  const double* wt1 = T1 == 1 ? (ENR ? tab + L.wy : tab + L.w) : tab + L.w;
  const double* wt2 = T2 == 1 ? (ENR ? tab + L.wy : tab + L.w) : tab + L.w;
  const double* ndo = tab + (S ? L.nd1 : L.nd0);   // own face at xi_D = S
  const double* ndn = tab + (S ? L.nd0 : L.nd1);   // neighbour's face at 1 - S

  T* lay = s_big;
  T* tr = lay + Sh::LAY;
  T* fl = tr + Sh::TR;

  // neighbour
  int nidx[3] = {ex, ey, ez};
  const int nmax[3] = {M.nx, M.ny, M.nz};
  nidx[D] += S ? 1 : -1;
  bool wall = false;
  if (nidx[D] < 0 || nidx[D] >= nmax[D]) {
    if (D == 1 && !M.fully_periodic) wall = true;
    nidx[D] = (nidx[D] + nmax[D]) % nmax[D];
  }
  const int64_t enb = nidx[0] + (int64_t)M.nx * (nidx[1] + (int64_t)M.ny * nidx[2]);
  const int64_t enr_nb = wall ? -1 : enr_index(M, nidx[0], nidx[1], nidx[2]);
  const T hown[3] = {hx, hy, hz};
  const T hd = hown[D];
  const T hdn = (D == 1) ? T(M.hy[nidx[1]]) : hd;
  const T ht1 = hown[T1], ht2 = hown[T2];
  const T tauF = wall ? T(M.pen * M.wall_mult) / hd : T(M.pen) * (T(1) / hd > T(1) / hdn ? T(1) / hd : T(1) / hdn);

  // Phase A: node layers on the face (value and normal derivative), both sides
  for (int t = tid; t < 2 * 3 * NP2; t += nt) {
    const int side = t / (3 * NP2), rem = t - side * 3 * NP2;
    const int c = rem / NP2, k = rem - c * NP2;
    if (side == 1 && wall) continue;
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
      const T x = side == 0 ? s_u[c * NP3 + B] : u[(enb * 3 + c) * NP3 + B];
      der += T(nd[l]) * x;
      if (l == lface) val = x;
    }
    lay[((side * 3 + c) * 2 + 0) * NP2 + k] = val;
    lay[((side * 3 + c) * 2 + 1) * NP2 + k] = der / (side == 0 ? hd : hdn);
  }
  __syncthreads();

  // Phase B: traces at the face Gauss points
  for (int t = tid; t < 2 * 3 * FP; t += nt) {
    const int side = t / (3 * FP), rem = t - side * 3 * FP;
    const int c = rem / FP, pt = rem - c * FP;
    if (side == 1 && wall) continue;
    const int q1 = pt % Q1, q2 = pt / Q1;
    const T* lv = lay + ((side * 3 + c) * 2 + 0) * NP2;
    const T* ln = lay + ((side * 3 + c) * 2 + 1) * NP2;
    T v = 0, d1 = 0, d2 = 0, dn = 0;
#pragma unroll
    for (int i2 = 0; i2 < NP; ++i2) {
      T av = 0, ad = 0, an = 0;
#pragma unroll
      for (int i1 = 0; i1 < NP; ++i1) {
        const T x = lv[i1 + NP * i2];
        av += T(St1[q1 * NP + i1]) * x;
        ad += T(Sdt1[q1 * NP + i1]) * x;
        an += T(St1[q1 * NP + i1]) * ln[i1 + NP * i2];
      }
      const T s2 = T(St2[q2 * NP + i2]), sd2 = T(Sdt2[q2 * NP + i2]);
      v += s2 * av;
      d1 += s2 * ad;
      d2 += sd2 * av;
      dn += s2 * an;
    }
    T* o = tr + (side * 3 + c) * 4 * Sh::FMAX;
    o[0 * Sh::FMAX + pt] = v;
    o[1 * Sh::FMAX + pt] = d1 / ht1;
    o[2 * Sh::FMAX + pt] = d2 / ht2;
    o[3 * Sh::FMAX + pt] = dn;
  }
  __syncthreads();

  // Phase C: numerical flux at each face point
  const T nu = T(M.nu), theta = T(M.theta);
  const T sg = S ? T(1) : T(-1);
  for (int pt = tid; pt < FP; pt += nt) {
    const int q1 = pt % Q1, q2 = pt / Q1;
    T um[3], up[3], gm[3][3], gp[3][3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const T* o = tr + (0 * 3 + c) * 4 * Sh::FMAX;
      um[c] = o[pt];
      gm[c][T1] = o[Sh::FMAX + pt];
      gm[c][T2] = o[2 * Sh::FMAX + pt];
      gm[c][D] = o[3 * Sh::FMAX + pt];
    }
    T psim = 0, gpsim[3] = {0, 0, 0};
    if (ENR) {
      const double* ps = M.psi + ((size_t)enr * M.psi_pts + M.psi_off[1 + 2 * D + S] + pt) * 4;
      psim = T(ps[0]);
      gpsim[0] = T(ps[1]);
      gpsim[1] = T(ps[2]);
      gpsim[2] = T(ps[3]);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        um[c] += psim * s_ut[c];
#pragma unroll
        for (int k = 0; k < 3; ++k) gm[c][k] += s_ut[c] * gpsim[k];
      }
    }
    if (wall) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        up[c] = -um[c];
#pragma unroll
        for (int k = 0; k < 3; ++k) gp[c][k] = gm[c][k];
      }
    } else {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const T* o = tr + (1 * 3 + c) * 4 * Sh::FMAX;
        up[c] = o[pt];
        gp[c][T1] = o[Sh::FMAX + pt];
        gp[c][T2] = o[2 * Sh::FMAX + pt];
        gp[c][D] = o[3 * Sh::FMAX + pt];
      }
      if (enr_nb >= 0) {
        const double* ps = M.psi + ((size_t)enr_nb * M.psi_pts + M.psi_off[1 + 2 * D + (1 - S)] + pt) * 4;
        const T psip = T(ps[0]);
        const T gpp[3] = {T(ps[1]), T(ps[2]), T(ps[3])};
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const T ut = u[M.enr_off + enr_nb * 3 + c];
          up[c] += psip * ut;
#pragma unroll
          for (int k = 0; k < 3; ++k) gp[c][k] += ut * gpp[k];
        }
      }
    }
    // n = sg e_D
    const T unm = sg * um[D], unp = sg * up[D];
    const T am = unm < 0 ? -unm : unm, ap = unp < 0 ? -unp : unp;
    const T lam = T(2) * (am > ap ? am : ap);
    const T wf = T(wt1[q1]) * T(wt2[q2]) * ht1 * ht2;
    T jmp[3], fv[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) jmp[c] = um[c] - up[c];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      // {{2 nu eps(u)}} n = nu/2 (grad u- + grad u-^T + grad u+ + grad u+^T) n
      const T visc = (gm[c][D] + gm[D][c] + gp[c][D] + gp[D][c]) * sg;
      fv[c] = T(0.5) * (um[c] * unm + up[c] * unp) + T(0.5) * lam * jmp[c] - T(0.5) * nu * visc +
              tauF * nu * jmp[c];
      fl[c * Sh::FMAX + pt] = wf * fv[c];
    }
    // F_g = -theta nu sym(jmp (x) n): entries [c][k] = -theta nu/2 (jmp_c n_k + jmp_k n_c)
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const T nk = (k == D) ? sg : T(0), nc = (c == D) ? sg : T(0);
        const T Fg = -theta * nu * T(0.5) * (jmp[c] * nk + jmp[k] * nc);
        fl[(3 + 3 * c + k) * Sh::FMAX + pt] = wf * Fg;
        if (ENR) rt[c] += wf * Fg * gpsim[k];
      }
    if (ENR)
#pragma unroll
      for (int c = 0; c < 3; ++c) rt[c] += wf * psim * fv[c];
  }
  __syncthreads();

  // Phase D: integrate against the own test functions (transpose of A/B)
  for (int t = tid; t < 3 * NP2; t += nt) {
    const int c = t / NP2, k = t - c * NP2;
    const int i1 = k % NP, i2 = k / NP;
    const T* fvc = fl + c * Sh::FMAX;
    const T* ft1 = fl + (3 + 3 * c + T1) * Sh::FMAX;
    const T* ft2 = fl + (3 + 3 * c + T2) * Sh::FMAX;
    const T* fnn = fl + (3 + 3 * c + D) * Sh::FMAX;
    T rv = 0, bn = 0;
#pragma unroll
    for (int q2 = 0; q2 < Q2; ++q2) {
      T a0 = 0, a1 = 0, a2 = 0, a3 = 0;
#pragma unroll
      for (int q1 = 0; q1 < Q1; ++q1) {
        const int pt = q1 + Q1 * q2;
        const T s1 = T(St1[q1 * NP + i1]), sd1 = T(Sdt1[q1 * NP + i1]);
        a0 += s1 * fvc[pt];
        a1 += sd1 * ft1[pt];
        a2 += s1 * ft2[pt];
        a3 += s1 * fnn[pt];
      }
      const T s2 = T(St2[q2 * NP + i2]), sd2 = T(Sdt2[q2 * NP + i2]);
      rv += s2 * (a0 + a1 / ht1) + sd2 * a2 / ht2;
      bn += s2 * a3;
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
      s_r[c * NP3 + B] += add;
    }
  }
  __syncthreads();
}

template <typename T, int NP, int NQ, int NQY, bool ENR>
__global__ __launch_bounds__(256) void vel_kernel(const MeshDev M, const T* __restrict__ u, T* __restrict__ r,
                                                  int layer_lo, int nlayers) {
  using Sh = VelShape<T, NP, NQ, NQY>;
  constexpr TabLayout L = tab_layout(NP, NQ, NQY);
  constexpr int NP3 = Sh::NP3, NPTS = Sh::NPTS;
  __shared__ T s_u[3 * NP3];
  __shared__ T s_r[3 * NP3];
  __shared__ T s_big[Sh::BIG];
  __shared__ T s_ut[3];
  __shared__ T s_red[3 * 4];
  const int tid = threadIdx.x, nt = blockDim.x;

  const int b = blockIdx.x;
  const int ex = b % M.nx;
  const int t0 = b / M.nx;
  int ey, ez;
  int64_t enr = -1;
  if (ENR) {
    const int slot = t0 % M.nslots;
    ez = t0 / M.nslots;
    ey = (slot == M.lower_slot) ? 0 : M.ny - 1;
    enr = b;
  } else {
    ey = layer_lo + t0 % nlayers;
    ez = t0 / nlayers;
  }
  const int64_t e = ex + (int64_t)M.nx * (ey + (int64_t)M.ny * ez);
  const T hx = T(M.hx), hz = T(M.hz), hy = T(M.hy[ey]);

  const double* tab = M.tab;
  const double* Sx = tab + L.S;
  const double* Dx = tab + L.D;
  const double* wx = tab + L.w;
  const double* Sy = ENR ? tab + L.Sy : tab + L.S;
  const double* Dy = ENR ? tab + L.Dy : tab + L.D;
  const double* wy = ENR ? tab + L.wy : tab + L.w;

  for (int i = tid; i < 3 * NP3; i += nt) s_u[i] = u[e * 3 * NP3 + i];
  if (ENR && tid < 3) s_ut[tid] = u[M.enr_off + enr * 3 + tid];
  __syncthreads();

  T* s_val = s_big;             // [c][pt]
  T* s_grad = s_big + 3 * NPTS; // [c][d][pt]
  // values at the Gauss points: x, y, z interpolation sweeps
  {
    T* tA = s_grad;                       // (NQ, NP, NP) x 3
    T* tB = tA + 3 * NQ * NP * NP;        // (NQ, NQY, NP) x 3
    sweep<0, NP, NP, NP, NQ, false, false>(s_u, NP3, tA, NQ * NP * NP, Sx, T(1), 3);
    __syncthreads();
    sweep<1, NQ, NP, NP, NQY, false, false>(tA, NQ * NP * NP, tB, NQ * NQY * NP, Sy, T(1), 3);
    __syncthreads();
    sweep<2, NQ, NQY, NP, NQ, false, false>(tB, NQ * NQY * NP, s_val, NPTS, Sx, T(1), 3);
    __syncthreads();
  }
  // gradients by collocation through the Gauss points
  sweep<0, NQ, NQY, NQ, NQ, false, false>(s_val, NPTS, s_grad + 0 * NPTS, 3 * NPTS, Dx, T(1) / hx, 3);
  sweep<1, NQ, NQY, NQ, NQY, false, false>(s_val, NPTS, s_grad + 1 * NPTS, 3 * NPTS, Dy, T(1) / hy, 3);
  sweep<2, NQ, NQY, NQ, NQ, false, false>(s_val, NPTS, s_grad + 2 * NPTS, 3 * NPTS, Dx, T(1) / hz, 3);
  __syncthreads();

  // pointwise flux G = 2 nu eps(u) - u (x) u, times the quadrature weight
  T rt[3] = {0, 0, 0};
  const T nu = T(M.nu);
  const T vol = hx * hy * hz;
  for (int pt = tid; pt < NPTS; pt += nt) {
    const int qx = pt % NQ, qy = (pt / NQ) % NQY, qz = pt / (NQ * NQY);
    const T wq = T(wx[qx]) * T(wy[qy]) * T(wx[qz]) * vol;
    T uu[3], gg[3][3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      uu[c] = s_val[c * NPTS + pt];
#pragma unroll
      for (int d = 0; d < 3; ++d) gg[c][d] = s_grad[(c * 3 + d) * NPTS + pt];
    }
    T gps[3] = {0, 0, 0};
    if (ENR) {
      const double* ps = M.psi + ((size_t)enr * M.psi_pts + pt) * 4;
      const T psv = T(ps[0]);
      gps[0] = T(ps[1]);
      gps[1] = T(ps[2]);
      gps[2] = T(ps[3]);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        uu[c] += psv * s_ut[c];
#pragma unroll
        for (int d = 0; d < 3; ++d) gg[c][d] += s_ut[c] * gps[d];
      }
    }
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const T G = wq * (nu * (gg[c][d] + gg[d][c]) - uu[c] * uu[d]);
        s_grad[(c * 3 + d) * NPTS + pt] = G;
        if (ENR) rt[c] += G * gps[d];
      }
  }
  __syncthreads();

  // integrate: W = sum_d D_d^T G_d / h_d, then transposed interpolation
  sweep<0, NQ, NQY, NQ, NQ, true, false>(s_grad + 0 * NPTS, 3 * NPTS, s_val, NPTS, Dx, T(1) / hx, 3);
  __syncthreads();
  sweep<1, NQ, NQY, NQ, NQY, true, true>(s_grad + 1 * NPTS, 3 * NPTS, s_val, NPTS, Dy, T(1) / hy, 3);
  __syncthreads();
  sweep<2, NQ, NQY, NQ, NQ, true, true>(s_grad + 2 * NPTS, 3 * NPTS, s_val, NPTS, Dx, T(1) / hz, 3);
  __syncthreads();
  {
    T* tB = s_grad;                       // (NQ, NQY, NP) x 3
    T* tA = tB + 3 * NQ * NQY * NP;       // (NQ, NP, NP) x 3
    sweep<2, NQ, NQY, NQ, NP, true, false>(s_val, NPTS, tB, NQ * NQY * NP, Sx, T(1), 3);
    __syncthreads();
    sweep<1, NQ, NQY, NP, NP, true, false>(tB, NQ * NQY * NP, tA, NQ * NP * NP, Sy, T(1), 3);
    __syncthreads();
    sweep<0, NQ, NP, NP, NP, true, false>(tA, NQ * NP * NP, s_r, NP3, Sx, T(1), 3);
    __syncthreads();
  }

  // faces
  vel_face<T, NP, NQ, NQY, ENR, 0, 0>(M, u, s_u, s_r, s_big, s_ut, ex, ey, ez, enr, hx, hy, hz, rt);
  vel_face<T, NP, NQ, NQY, ENR, 0, 1>(M, u, s_u, s_r, s_big, s_ut, ex, ey, ez, enr, hx, hy, hz, rt);
  vel_face<T, NP, NQ, NQY, ENR, 1, 0>(M, u, s_u, s_r, s_big, s_ut, ex, ey, ez, enr, hx, hy, hz, rt);
  vel_face<T, NP, NQ, NQY, ENR, 1, 1>(M, u, s_u, s_r, s_big, s_ut, ex, ey, ez, enr, hx, hy, hz, rt);
  vel_face<T, NP, NQ, NQY, ENR, 2, 0>(M, u, s_u, s_r, s_big, s_ut, ex, ey, ez, enr, hx, hy, hz, rt);
  vel_face<T, NP, NQ, NQY, ENR, 2, 1>(M, u, s_u, s_r, s_big, s_ut, ex, ey, ez, enr, hx, hy, hz, rt);

  for (int i = tid; i < 3 * NP3; i += nt) r[e * 3 * NP3 + i] = s_r[i];
  if (ENR) {
    block_sum3(rt, s_red);
    if (tid < 3) r[M.enr_off + enr * 3 + tid] = rt[0];
  }
}

template <typename T, int NP, int NQ, int NQW>
int launch_vel_t(const dg_mesh* m, const MeshDev& M, const void* u, void* r, hipStream_t s) {
  const T* uu = static_cast<const T*>(u);
  T* rr = static_cast<T*>(r);
  const int lo = (m->P.fully_periodic || m->lower_slot < 0) ? 0 : 1;
  const int hi = (m->P.fully_periodic || m->upper_slot < 0) ? m->P.ny - 1 : m->P.ny - 2;
  const int nl = hi - lo + 1;
  if (nl > 0) {
    const unsigned nb = (unsigned)((int64_t)m->P.nx * nl * m->P.nz);
    hipLaunchKernelGGL((vel_kernel<T, NP, NQ, NQ, false>), dim3(nb), dim3(256), 0, s, M, uu, rr, lo, nl);
  }
  if (m->nenr > 0) {
    hipLaunchKernelGGL((vel_kernel<T, NP, NQ, NQW, true>), dim3((unsigned)m->nenr), dim3(256), 0, s, M, uu, rr,
                       0, 0);
  }
  return check_hip(hipGetLastError(), "velocity kernel launch");
}

MeshDev make_meshdev_u(const dg_mesh* m) {
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
  M.tab = m->tab_u;
  M.psi = m->psi;
  M.psi_pts = m->psi_pts;
  for (int f = 0; f <= 6; ++f) M.psi_off[f] = (f == 0) ? 0 : psi_face_offset(m->P.nq_u, m->P.nq_wn, f - 1);
  M.nu = m->P.nu;
  M.theta = m->P.theta;
  M.pen = m->P.ip_factor_u * (m->P.k_u + 1.0) * (m->P.k_u + 1.0);
  M.wall_mult = m->P.wall_ip_mult;
  M.enr_off = m->ncell * 3 * (int64_t)m->np_u * m->np_u * m->np_u;
  return M;
}

}  // namespace

// (np, nq, nq_wn) combinations compiled in.
#define DG_VEL_COMBOS(X) \
  X(3, 4, 8)             \
  X(3, 4, 4)             \
  X(4, 4, 8)             \
  X(4, 5, 8)             \
  X(4, 5, 5)             \
  X(5, 7, 8)             \
  X(6, 8, 8)

bool velocity_supported(int np, int nq, int nqy) {
#define X(a, b, c) \
  if (np == a && nq == b && nqy == c) return true;
  DG_VEL_COMBOS(X)
#undef X
  return false;
}

const char* velocity_combos() { return "velocity (k+1, nq_u, nq_wn): (3,4,8) (3,4,4) (4,4,8) (4,5,8) (4,5,5) (5,7,8) (6,8,8)"; }

int launch_velocity(const dg_mesh* m, dg_prec prec, const void* u, void* r, hipStream_t s) {
  const MeshDev M = make_meshdev_u(m);
  const int np = m->np_u, nq = m->P.nq_u, nqw = m->P.nq_wn;
  // without enriched cells only the regular kernel runs: nq_wn is irrelevant
#define X(a, b, c)                                                                 \
  if (np == a && nq == b && (nqw == c || m->nenr == 0)) {                          \
    return prec == DG_F64 ? launch_vel_t<double, a, b, c>(m, M, u, r, s)           \
                          : launch_vel_t<float, a, b, c>(m, M, u, r, s);           \
  }
  DG_VEL_COMBOS(X)
#undef X
  return set_error(DG_ERR_UNSUPPORTED, "velocity degree/quadrature combination not compiled");
}

}  // namespace dgwm
