// SIP Poisson operator (arXiv 1705.08813, Sec. 4.2, pressure Laplace term
// with flux eq. ipflux and homogeneous Neumann walls), matrix-free:
//   (A p)(q) = sum_e (grad q, grad p)_e
//            + sum_F [ -1/2 (grad q.n)(p- - p+) - q ({{grad p}}.n - tau_F (p- - p+)) ]_F
// and the Jacobi diagonal of A.  Box (affine) meshes.
//
// One workgroup per cell, sum-factorized volume term, element-by-element
// face terms (each cell reads its neighbour's nodal values), single writer
// per output entry.
#include <algorithm>

#include "batch.h"

namespace dgwm {

namespace {

// Neighbour of cell e = (ex, ey, ez) across face (D, S): -1 for a (Neumann)
// wall.  Cell counts stay below 2^31 (checked at set-up).
__device__ __forceinline__ int poi_nb(const MeshDev& M, int e, int ex, int ey, int ez, int D, int S) {
  const int j = D == 0 ? ex : (D == 1 ? ey : ez);
  const int nmax = D == 0 ? M.nx : (D == 1 ? M.ny : M.nz);
  const int step = D == 0 ? 1 : (D == 1 ? M.nx : M.nx * M.ny);
  if (S ? j == nmax - 1 : j == 0) {
    if (D == 1 && !M.fully_periodic) return -1;
    return S ? e - (nmax - 1) * step : e + (nmax - 1) * step;
  }
  return S ? e + step : e - step;
}

// Cells per workgroup: one thread per pencil (line of NP nodes), so a cell
// uses NP^2 threads and a 256-thread workgroup holds 256 / NP^2 cells.
template <int NP>
struct PoiBlk {
  static constexpr int NP2 = NP * NP, NP3 = NP2 * NP;
  static constexpr int CB = 256 / NP2 > 0 ? 256 / NP2 : 1;
  static constexpr int NT = CB * NP2;
};

// Pencil through tangential node (a, b) along direction D: first node and stride.
template <int NP>
__device__ __forceinline__ int pencil_base(int D, int a, int b) {
  return D == 0 ? NP * (a + NP * b) : (D == 1 ? a + NP * NP * b : a + NP * b);
}
template <int NP>
__device__ __forceinline__ constexpr int pencil_stride(int D) {
  return D == 0 ? 1 : (D == 1 ? NP : NP * NP);
}

// LDS layout of one cell: node (i, j, k) at i + SJ j + SK k, cells SC apart.
// The padding spreads the pencils that one wavefront reads or writes in the
// same instruction (16 threads of a cell, one node each, along x, y or z)
// over the LDS banks; the unpadded layout maps the NP = 4 pencils onto a
// quarter of the banks.
template <int NP>
struct PoiLds {
  static constexpr int SJ = NP, SK = NP * NP + (NP == 4 ? 1 : 0), SC = NP == 4 ? 76 : NP * NP * NP;
  static __device__ __forceinline__ int base(int D, int a, int b) {
    return D == 0 ? SJ * a + SK * b : (D == 1 ? a + SK * b : a + SJ * b);
  }
  static __device__ __forceinline__ constexpr int stride(int D) { return D == 0 ? 1 : (D == 1 ? SJ : SK); }
};

// Poisson operator on box cells.  On an affine box cell every term
// separates: with the reference mass M and stiffness K of the 1-D basis
// (built with the operator's Gauss rule, hence identical to quadrature),
//   cell:   (hy hz/hx) Mz My Kx + (hx hz/hy) Mz Ky Mx + (hx hy/hz) Kz My Mx
//   face D: (area) M_t1 M_t2 applied to a face source s_D that lives on the
//           pencils along D: for the face at xi_D = s with outward sign sg,
//           jump J = p- - p+ and G = tau J - sg {{dp/dx_D}},
//           s_D(l) += -1/2 sg N_l'(s)/h_D J + [l is the face node] G.
// Writing Q_D = (area_D/h_D) K_D p + area_D s_D (pencil-local along D),
//   A p = Mx (My Qz + Mz Qy) + My Mz Qx,
// evaluated as z-, y-, x-sweeps over LDS.  Each thread owns one pencil of
// every direction of its cell and reads the six neighbour pencils it needs
// for the traces straight from global memory (no atomics: every output has
// one writer).
// The cells of block blk: [blk CB, (blk + 1) CB).
template <typename T, int NP, int KIND>
__device__ __forceinline__ void poisson_body(const MeshDev& M, const T* __restrict__ p, T* __restrict__ y,
                                             int64_t ncell, int blk, const PoiEpi<T>& E) {
  using BL = PoiBlk<NP>;
  constexpr int NP2 = BL::NP2, NP3 = BL::NP3, CB = BL::CB;
  using LD = PoiLds<NP>;
  // In FP64 the input P and Q_x share one array (P is read into registers
  // first, one more barrier) so that five workgroups fit in a CU's LDS; FP32
  // keeps a separate input array.
  constexpr bool kAlias = sizeof(T) == 8;
  __shared__ T s_X[CB * LD::SC];
  __shared__ T s_Y[CB * LD::SC];
  __shared__ T s_Z[CB * LD::SC];
  __shared__ T s_P[kAlias ? 1 : CB * LD::SC];

  const int tid = threadIdx.x;
  const int c = tid / NP2, t = tid - c * NP2;
  const int a = t % NP, b = t / NP;
  const int64_t e = (int64_t)blk * CB + c;
  const bool live = tid < BL::NT && e < ncell;
  // the kind is a template argument so that the plain operator keeps no
  // registers for the epilogue operands
  constexpr bool pre = KIND == kChebFirst;

  constexpr PoiOps O = poi_ops(NP);
  const T* ops = sizeof(T) == 8 ? reinterpret_cast<const T*>(M.tab + M.ops_off)
                                : reinterpret_cast<const T*>(M.tab + M.ops_off + O.f32);
  const T* Mm = ops + O.M;
  const T* Km = ops + O.K;
  const T* nd0 = ops + O.nd0;
  const T* nd1 = ops + O.nd1;

  T* sX = s_X + c * LD::SC;
  T* sY = s_Y + c * LD::SC;
  T* sZ = s_Z + c * LD::SC;
  T* sP = kAlias ? sX : s_P + c * LD::SC;

  T px[NP];
  T eb[NP], ei_[NP], ed[NP];  // epilogue operands b, dinv, d, loaded with the input
  T vnb[3][2], dnb[3][2], rnb[3][2];
  bool wall[3][2];
  T h[3], rh[3];
  if (live) {
    const int ei = (int)e;
    const int ex = ei % M.nx, eyz = ei / M.nx, ey = eyz % M.ny, ez = eyz / M.ny;
    h[0] = T(M.hx);
    h[1] = T(M.hy[ey]);
    h[2] = T(M.hz);
    rh[0] = T(M.ihx);
    rh[1] = T(M.ihy[ey]);
    rh[2] = T(M.ihz);
    const int bx = pencil_base<NP>(0, a, b);
    const int64_t o = e * NP3 + bx;
    if (KIND != kPlain) {
#pragma unroll
      for (int l = 0; l < NP; ++l) eb[l] = E.b[o + l];
    }
    if (KIND >= kCheb) {
#pragma unroll
      for (int l = 0; l < NP; ++l) ei_[l] = E.dinv[o + l];
    }
    if (KIND == kCheb && E.c1 != T(0)) {
#pragma unroll
      for (int l = 0; l < NP; ++l) ed[l] = E.zout[o + l];
    }
    if (pre) {  // p is b
#pragma unroll
      for (int l = 0; l < NP; ++l) px[l] = E.c0 * ei_[l] * eb[l];
    } else {
#pragma unroll
      for (int l = 0; l < NP; ++l) px[l] = p[o + l];
    }
#pragma unroll
    for (int l = 0; l < NP; ++l) sP[LD::base(0, a, b) + l] = px[l];
    // traces of the six neighbours on the shared faces: value and d/dx_D
#pragma unroll
    for (int D = 0; D < 3; ++D) {
      const int bD = pencil_base<NP>(D, a, b);
#pragma unroll
      for (int S = 0; S < 2; ++S) {
        const int nb = poi_nb(M, ei, ex, ey, ez, D, S);
        wall[D][S] = nb < 0;
        T v = 0, d = 0, rn = rh[D];
        if (nb >= 0) {
          const T* pn = p + (int64_t)nb * NP3 + bD;
          T q[NP];
#pragma unroll
          for (int l = 0; l < NP; ++l) q[l] = pn[l * pencil_stride<NP>(D)];
          if (pre) {
            const T* dn = E.dinv + (int64_t)nb * NP3 + bD;
#pragma unroll
            for (int l = 0; l < NP; ++l) q[l] *= E.c0 * dn[l * pencil_stride<NP>(D)];
          }
          // neighbour below (S = 0) meets us at its xi_D = 1, above (S = 1) at xi_D = 0
          const T* nd = S ? nd0 : nd1;
#pragma unroll
          for (int l = 0; l < NP; ++l) d += nd[l] * q[l];
          v = S ? q[0] : q[NP - 1];
          if (D == 1) {
            const int yn = S ? (ey + 1 == M.ny ? 0 : ey + 1) : (ey == 0 ? M.ny - 1 : ey - 1);
            rn = T(M.ihy[yn]);
          }
          d *= rn;
        }
        vnb[D][S] = v;
        dnb[D][S] = d;
        rnb[D][S] = rn;
      }
    }
  }
  __syncthreads();

  // the thread's y and z pencils of P
  T pyz[2][NP];
  if (live) {
#pragma unroll
    for (int D = 1; D < 3; ++D) {
      const int bD = LD::base(D, a, b);
#pragma unroll
      for (int l = 0; l < NP; ++l) pyz[D - 1][l] = sP[bD + l * LD::stride(D)];
    }
  }
  if (kAlias) __syncthreads();

  // Q_D on the thread's pencil of every direction
  if (live) {
    const T pen = T(M.pen);
#pragma unroll
    for (int D = 0; D < 3; ++D) {
      const int bD = LD::base(D, a, b);
      T x[NP];
#pragma unroll
      for (int l = 0; l < NP; ++l) x[l] = D == 0 ? px[l] : pyz[D - 1][l];
      const T rd = rh[D];
      const T area = D == 0 ? h[1] * h[2] : (D == 1 ? h[0] * h[2] : h[0] * h[1]);
      T d0 = 0, d1 = 0;
#pragma unroll
      for (int l = 0; l < NP; ++l) {
        d0 += nd0[l] * x[l];
        d1 += nd1[l] * x[l];
      }
      d0 *= rd;
      d1 *= rd;
      T J0 = 0, G0 = 0, J1 = 0, G1 = 0;
      if (!wall[D][0]) {  // face at xi_D = 0, outward sign -1
        const T tau = pen * (rd > rnb[D][0] ? rd : rnb[D][0]);
        J0 = x[0] - vnb[D][0];
        G0 = tau * J0 + T(0.5) * (d0 + dnb[D][0]);
      }
      if (!wall[D][1]) {  // face at xi_D = 1, outward sign +1
        const T tau = pen * (rd > rnb[D][1] ? rd : rnb[D][1]);
        J1 = x[NP - 1] - vnb[D][1];
        G1 = tau * J1 - T(0.5) * (d1 + dnb[D][1]);
      }
      const T cv = area * rd;
      T* dst = D == 0 ? sX : (D == 1 ? sY : sZ);
#pragma unroll
      for (int l = 0; l < NP; ++l) {
        T k = 0;
#pragma unroll
        for (int m = 0; m < NP; ++m) k += Km[l * NP + m] * x[m];
        T q = cv * (k + T(0.5) * nd0[l] * J0 - T(0.5) * nd1[l] * J1);
        if (l == 0) q += area * G0;
        if (l == NP - 1) q += area * G1;
        dst[bD + l * LD::stride(D)] = q;
      }
    }
  }
  __syncthreads();

  // z sweeps: Y <- Mz Qy, X <- Mz Qx
  if (live) {
    const int bz = LD::base(2, a, b);
    constexpr int sz = LD::SK;
    T u[NP], w[NP];
#pragma unroll
    for (int l = 0; l < NP; ++l) {
      u[l] = sY[bz + l * sz];
      w[l] = sX[bz + l * sz];
    }
#pragma unroll
    for (int l = 0; l < NP; ++l) {
      T su = 0, sw = 0;
#pragma unroll
      for (int m = 0; m < NP; ++m) {
        su += Mm[l * NP + m] * u[m];
        sw += Mm[l * NP + m] * w[m];
      }
      sY[bz + l * sz] = su;
      sX[bz + l * sz] = sw;
    }
  }
  __syncthreads();

  // y sweeps: Z <- My Qz + Y, X <- My X
  if (live) {
    const int by = LD::base(1, a, b);
    constexpr int sy = LD::SJ;
    T u[NP], w[NP], v[NP];
#pragma unroll
    for (int l = 0; l < NP; ++l) {
      u[l] = sZ[by + l * sy];
      v[l] = sY[by + l * sy];
      w[l] = sX[by + l * sy];
    }
#pragma unroll
    for (int l = 0; l < NP; ++l) {
      T su = v[l], sw = 0;
#pragma unroll
      for (int m = 0; m < NP; ++m) {
        su += Mm[l * NP + m] * u[m];
        sw += Mm[l * NP + m] * w[m];
      }
      sZ[by + l * sy] = su;
      sX[by + l * sy] = sw;
    }
  }
  __syncthreads();

  // x sweep and write-out: y = Mx Z + X
  if (live) {
    const int bx = pencil_base<NP>(0, a, b);
    const int lx = LD::base(0, a, b);
    T u[NP];
#pragma unroll
    for (int l = 0; l < NP; ++l) u[l] = sZ[lx + l];
    const int64_t o = e * NP3 + bx;
#pragma unroll
    for (int l = 0; l < NP; ++l) {
      T s = sX[lx + l];
#pragma unroll
      for (int m = 0; m < NP; ++m) s += Mm[l * NP + m] * u[m];
      if (KIND == kPlain) {
        y[o + l] = s;
      } else if (KIND == kResid) {
        y[o + l] = eb[l] - s;
      } else {
        T v = E.c2 * ei_[l] * (eb[l] - s);
        if (E.c1 != T(0)) v += E.c1 * (pre ? px[l] : px[l] - ed[l]);
        if (pre) E.z1[o + l] = px[l];
        E.zout[o + l] = px[l] + v;
      }
    }
  }
}

template <typename T, int NP, int KIND>
__global__ __launch_bounds__(256) void poisson_kernel(const MeshDev M, const T* __restrict__ p, T* __restrict__ y,
                                                      int64_t ncell, int nblocks, int64_t vstride,
                                                      const PoiEpi<T> E) {
  // blockIdx.y selects one of several vectors stored vstride apart
  p += blockIdx.y * vstride;
  y += blockIdx.y * vstride;
  // contiguous cell ranges per XCD (workgroups are dealt round-robin over 8)
  const int bid = blockIdx.x;
  const int q8 = nblocks >> 3, r8 = nblocks & 7, xcd = bid & 7, m8 = bid >> 3;
  const int blk = xcd * q8 + (xcd < r8 ? xcd : r8) + m8;
  poisson_body<T, NP, KIND>(M, p, y, ncell, blk, E);
}

// One launch over the segments of up to kPoiSegs meshes (cells of each
// segment in order; small meshes, so no XCD remapping).
template <typename T, int NP, int KIND>
__global__ __launch_bounds__(256) void poisson_kernel_batched(const SegArr<PoiSeg<T>, kPoiSegs> a) {
  const int si = find_seg(a, (int64_t)blockIdx.x);
  const PoiSeg<T>& S = a.s[si];
  poisson_body<T, NP, KIND>(S.M, S.p, S.y, S.ncell, (int)((int64_t)blockIdx.x - S.blk0), S.E);
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

}  // namespace

#define DG_POI_COMBOS(X) X(2, 2) X(3, 3) X(4, 4) X(5, 5) X(6, 6)

// Mesh arguments of multigrid level l (level 0: the mesh itself).
MeshDev poisson_meshdev(const dg_mesh* m, int l) {
  MeshDev M{};
  const MgLevel* lv = (l > 0) ? &m->mg[l] : nullptr;
  M.nx = lv ? lv->nx : m->P.nx;
  M.ny = lv ? lv->ny : m->P.ny;
  M.nz = lv ? lv->nz : m->P.nz;
  M.fully_periodic = m->P.fully_periodic;
  M.lower_slot = m->lower_slot;
  M.upper_slot = m->upper_slot;
  M.nslots = m->n_enr_layers;
  M.hx = lv ? lv->hx : m->hx;
  M.hz = lv ? lv->hz : m->hz;
  M.hy = lv ? lv->hy : m->hy;
  M.ihy = M.hy + M.ny;
  M.ihx = 1.0 / M.hx;
  M.ihz = 1.0 / M.hz;
  M.tab = m->tab_p;
  M.ops_off = tab_layout(m->np_p, m->P.nq_p, m->P.nq_p).size;
  M.pen = m->P.ip_factor_p * (m->P.k_p + 1.0) * (m->P.k_p + 1.0);
  return M;
}

namespace {
MeshDev make_meshdev_p(const dg_mesh* m, int l = 0) { return poisson_meshdev(m, l); }
}  // namespace

int poisson_cells_per_block(int np) {
  switch (np) {
    case 2: return PoiBlk<2>::CB;
    case 3: return PoiBlk<3>::CB;
    case 4: return PoiBlk<4>::CB;
    case 5: return PoiBlk<5>::CB;
    case 6: return PoiBlk<6>::CB;
  }
  return 0;
}

template <typename T>
int launch_poisson_batched(int np, int kind, const PoiSeg<T>* segs, int nseg, hipStream_t s) {
  const int cb = poisson_cells_per_block(np);
  if (cb <= 0) return set_error(DG_ERR_UNSUPPORTED, "poisson degree not compiled");
  for (int c0 = 0; c0 < nseg; c0 += kPoiSegs) {
    SegArr<PoiSeg<T>, kPoiSegs> a{};
    a.n = std::min(kPoiSegs, nseg - c0);
    int64_t blk = 0;
    for (int i = 0; i < a.n; ++i) {
      a.s[i] = segs[c0 + i];
      a.s[i].blk0 = blk;
      blk += (a.s[i].ncell + cb - 1) / cb;
    }
    if (blk == 0) continue;
    const dim3 g((unsigned)blk);
    bool done = false;
#define X(q, b)                                                                                               \
    if (np == q) {                                                                                            \
      done = true;                                                                                            \
      switch (kind) {                                                                                         \
        case kPlain: hipLaunchKernelGGL((poisson_kernel_batched<T, q, kPlain>), g, dim3(256), 0, s, a); break; \
        case kResid: hipLaunchKernelGGL((poisson_kernel_batched<T, q, kResid>), g, dim3(256), 0, s, a); break; \
        case kCheb: hipLaunchKernelGGL((poisson_kernel_batched<T, q, kCheb>), g, dim3(256), 0, s, a); break;   \
        default: hipLaunchKernelGGL((poisson_kernel_batched<T, q, kChebFirst>), g, dim3(256), 0, s, a);        \
      }                                                                                                       \
    }
    DG_POI_COMBOS(X)
#undef X
    if (!done) return set_error(DG_ERR_UNSUPPORTED, "poisson degree not compiled");
    if (int rc = check_hip(hipGetLastError(), "batched poisson kernel launch")) return rc;
  }
  return DG_OK;
}
template int launch_poisson_batched<double>(int, int, const PoiSeg<double>*, int, hipStream_t);
template int launch_poisson_batched<float>(int, int, const PoiSeg<float>*, int, hipStream_t);

bool poisson_supported(int np, int nq) {
#define X(a, b) \
  if (np == a && nq == b) return true;
  DG_POI_COMBOS(X)
#undef X
  return false;
}

const char* poisson_combos() { return "poisson (k+1, nq_p): (2,2) (3,3) (4,4) (5,5) (6,6)"; }

template <typename T>
static int launch_poisson_t(const dg_mesh* m, int l, const T* p, T* y, hipStream_t s, int nvec, int64_t vstride,
                     const PoiEpi<T>& E) {
  const MeshDev M = make_meshdev_p(m, l);
  const int64_t ncell = l > 0 ? m->mg[l].ncell : m->ncell;
#define X(a, b)                                                                                           \
  if (m->np_p == a && m->P.nq_p == b) {                                                                   \
    const int nb = (int)((ncell + PoiBlk<a>::CB - 1) / PoiBlk<a>::CB);                                    \
    switch (E.kind) {                                                                                     \
      case kPlain:                                                                                        \
        hipLaunchKernelGGL((poisson_kernel<T, a, kPlain>), dim3(nb, nvec), dim3(256), 0, s, M, p, y, ncell, \
                           nb, vstride, E);                                                               \
        break;                                                                                            \
      case kResid:                                                                                        \
        hipLaunchKernelGGL((poisson_kernel<T, a, kResid>), dim3(nb, nvec), dim3(256), 0, s, M, p, y, ncell, \
                           nb, vstride, E);                                                               \
        break;                                                                                            \
      case kCheb:                                                                                         \
        hipLaunchKernelGGL((poisson_kernel<T, a, kCheb>), dim3(nb, nvec), dim3(256), 0, s, M, p, y, ncell,  \
                           nb, vstride, E);                                                               \
        break;                                                                                            \
      default:                                                                                            \
        hipLaunchKernelGGL((poisson_kernel<T, a, kChebFirst>), dim3(nb, nvec), dim3(256), 0, s, M, p, y,    \
                           ncell, nb, vstride, E);                                                        \
    }                                                                                                     \
    return check_hip(hipGetLastError(), "poisson kernel launch");                                         \
  }
  DG_POI_COMBOS(X)
#undef X
  return set_error(DG_ERR_UNSUPPORTED, "poisson degree/quadrature combination not compiled");
}

int launch_poisson_level(const dg_mesh* m, int l, dg_prec prec, const void* p, void* y, hipStream_t s, int nvec,
                         int64_t vstride) {
  if (prec == DG_F64) {
    const PoiEpi<double> E{kPlain, nullptr, nullptr, nullptr, nullptr, 0.0, 0.0, 0.0};
    return launch_poisson_t<double>(m, l, static_cast<const double*>(p), static_cast<double*>(y), s, nvec, vstride,
                                    E);
  }
  const PoiEpi<float> E{kPlain, nullptr, nullptr, nullptr, nullptr, 0.0f, 0.0f, 0.0f};
  return launch_poisson_t<float>(m, l, static_cast<const float*>(p), static_cast<float*>(y), s, nvec, vstride, E);
}

template <typename T>
int launch_poisson_resid(const dg_mesh* m, int l, const T* x, const T* b, T* r, hipStream_t s) {
  const PoiEpi<T> E{kResid, b, nullptr, nullptr, nullptr, T(0), T(0), T(0)};
  return launch_poisson_t<T>(m, l, x, r, s, 1, 0, E);
}

template <typename T>
int launch_poisson_cheb(const dg_mesh* m, int l, const T* z, T* zout, const T* b, const T* dinv, T c1, T c2,
                        hipStream_t s) {
  const PoiEpi<T> E{kCheb, b, dinv, nullptr, zout, c1, c2, T(0)};
  return launch_poisson_t<T>(m, l, z, nullptr, s, 1, 0, E);
}

template <typename T>
int launch_poisson_cheb_first(const dg_mesh* m, int l, T c0, T* zout, T* z1, const T* b, const T* dinv, T c1, T c2,
                              hipStream_t s) {
  const PoiEpi<T> E{kChebFirst, b, dinv, z1, zout, c1, c2, c0};
  return launch_poisson_t<T>(m, l, b, nullptr, s, 1, 0, E);
}

template int launch_poisson_resid<double>(const dg_mesh*, int, const double*, const double*, double*, hipStream_t);
template int launch_poisson_resid<float>(const dg_mesh*, int, const float*, const float*, float*, hipStream_t);
template int launch_poisson_cheb<double>(const dg_mesh*, int, const double*, double*, const double*, const double*,
                                         double, double, hipStream_t);
template int launch_poisson_cheb<float>(const dg_mesh*, int, const float*, float*, const float*, const float*, float,
                                        float, hipStream_t);
template int launch_poisson_cheb_first<double>(const dg_mesh*, int, double, double*, double*, const double*,
                                               const double*, double, double, hipStream_t);
template int launch_poisson_cheb_first<float>(const dg_mesh*, int, float, float*, float*, const float*, const float*,
                                              float, float, hipStream_t);

int launch_poisson(const dg_mesh* m, dg_prec prec, const void* p, void* y, hipStream_t s) {
  return launch_poisson_level(m, 0, prec, p, y, s);
}

int launch_poisson_diag_level(const dg_mesh* m, int l, hipStream_t s) {
  const MeshDev M = make_meshdev_p(m, l);
  const int64_t ncell = l > 0 ? m->mg[l].ncell : m->ncell;
  const int64_t n = l > 0 ? m->mg[l].n : m->n_p;
  double* dg = l > 0 ? m->mg[l].diag : m->diag;
  float* dg32 = l > 0 ? m->mg[l].diag32 : m->diag32;
  const unsigned nb = (unsigned)((n + 255) / 256);
#define X(a, b)                                                                                           \
  if (m->np_p == a && m->P.nq_p == b) {                                                                   \
    hipLaunchKernelGGL((poisson_diag_kernel<a, b>), dim3(nb), dim3(256), 0, s, M, ncell, dg, dg32);       \
    return check_hip(hipGetLastError(), "poisson diagonal launch");                                       \
  }
  DG_POI_COMBOS(X)
#undef X
  return set_error(DG_ERR_UNSUPPORTED, "poisson degree/quadrature combination not compiled");
}

int launch_poisson_diag(const dg_mesh* m, hipStream_t s) { return launch_poisson_diag_level(m, 0, s); }

}  // namespace dgwm
