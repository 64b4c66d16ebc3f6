// Pressure gradient and velocity divergence terms of the dual-splitting
// scheme (arXiv 1705.08813, Sec. 4.2), FP64, flat (box) meshes.
//
//   P: g(v) = -(div v, p)_e + (v . n, {{p}})_{boundary of e}     (velocity test functions)
//   C: c(q) = -(grad q, u)_e + (q, {{u}} . n)_{boundary of e}    (pressure test functions)
//
// {{.}} the central average; on no-slip walls both terms take the interior
// value, p+ = p- and u+ = u- (the boundary conditions Sec. 4.2 gives for the
// pressure Poisson equation and the projection step).  u is the full velocity with
// psi u~ in enriched cells, and the velocity test functions include psi e_c
// (l = 0) or psi N_B e_c with the cell's eight trilinear vertex functions
// N_B, B = bx + 2 (by + 2 bz) (l = 1, Sec. 3.1 eq. enrichment; LE = 8
// enrichment functions per component, coefficients [c][B]).
// Both use the velocity quadrature of the cell (nq^3, nq x nqy x nq in
// enriched cells) and of its faces (x- and z-faces take the cell's
// wall-normal rule, which every neighbour in the same layer shares).
//
// One workgroup per cell; the output block of the cell is accumulated in LDS
// (volume term first, then the faces direction by direction) and written
// once, so every output has one writer.  Values at points come from
// sum-factorized interpolation sweeps, test-function integrals from the
// transposed sweeps (one thread per line, the 1-D tables of both bases at
// both rules as compile-time literals); faces interpolate the node layer at
// the face (the Gauss-Lobatto nodal basis has its face values on that layer)
// of the cell and of its neighbour.  All global reads of a cell, neighbour
// layers included, are issued before its first barrier.
#include "ctab.h"
#include "kern_common.h"

namespace dgwm {

namespace {

constexpr int kDgThreads = 256;

struct DgArgs {
  int nx, ny, nz, lower_slot, upper_slot, nslots, psi_pts, fully_periodic;
  int psi_off[7];          // volume, then the six faces f = 2d + s
  int64_t ncell;
  double hx, hz;
  const double* hy;        // ny heights
  const double* psi;       // [enr][psi_pts][4]
  const double* in;        // p (gradient) or u (divergence)
  double* out;
};

struct CellGeo {
  int ex, ey, ez;
  int64_t e, enr;          // enriched index or -1
  double h[3];
};

__device__ __forceinline__ int64_t enr_of(const DgArgs& A, int ex, int ey, int ez) {
  if (A.fully_periodic) return -1;
  int slot = -1;
  if (ey == 0 && A.lower_slot >= 0) slot = A.lower_slot;
  else if (ey == A.ny - 1 && A.upper_slot >= 0) slot = A.upper_slot;
  return slot < 0 ? -1 : ex + (int64_t)A.nx * (slot + (int64_t)A.nslots * ez);
}

// Cell of block b: regular cells b = ex + nx (ly + nlayers ez), ey = layer_lo
// + ly; enriched cells b = enriched index.
template <bool ENR>
__device__ __forceinline__ CellGeo cell_of_block(const DgArgs& A, int64_t b, int layer_lo, int nlayers) {
  CellGeo g;
  g.ex = (int)(b % A.nx);
  const int64_t t0 = b / A.nx;
  if (ENR) {
    const int slot = (int)(t0 % A.nslots);
    g.ez = (int)(t0 / A.nslots);
    g.ey = slot == A.lower_slot ? 0 : A.ny - 1;
  } else {
    g.ey = layer_lo + (int)(t0 % nlayers);
    g.ez = (int)(t0 / nlayers);
  }
  g.e = g.ex + (int64_t)A.nx * (g.ey + (int64_t)A.ny * g.ez);
  g.enr = ENR ? b : -1;
  g.h[0] = A.hx;
  g.h[1] = A.hy[g.ey];
  g.h[2] = A.hz;
  return g;
}

// Neighbour across face (d, s): cell index (and its indices), or -1 on a no-slip wall.
__device__ __forceinline__ int64_t neighbour(const DgArgs& A, const CellGeo& g, int d, int s, int& nx_, int& ny_,
                                             int& nz_) {
  int i[3] = {g.ex, g.ey, g.ez};
  const int n[3] = {A.nx, A.ny, A.nz};
  int j = i[d] + (s ? 1 : -1);
  if (j < 0 || j >= n[d]) {
    if (d == 1 && !A.fully_periodic) return -1;
    j = j < 0 ? j + n[d] : j - n[d];
  }
  i[d] = j;
  nx_ = i[0];
  ny_ = i[1];
  nz_ = i[2];
  return i[0] + (int64_t)A.nx * (i[1] + (int64_t)A.ny * i[2]);
}

// Node index of position (l1, l2) on the layer of face (d, s) of an NP^3
// nodal block (tangential directions t1 < t2).
template <int NP>
__device__ __forceinline__ int layer_node(int d, int s, int l1, int l2) {
  const int ld = s ? NP - 1 : 0;
  if (d == 0) return ld + NP * (l1 + NP * l2);
  if (d == 1) return l1 + NP * (ld + NP * l2);
  return l1 + NP * (l2 + NP * ld);
}

// Trilinear vertex function B at reference point (x0, x1, x2) and its
// reference derivatives d[3].
__device__ __forceinline__ double vtx(int B, const double x[3], double d[3]) {
  const double a0 = (B & 1) ? x[0] : 1.0 - x[0], a1 = (B & 2) ? x[1] : 1.0 - x[1], a2 = (B & 4) ? x[2] : 1.0 - x[2];
  const double s0 = (B & 1) ? 1.0 : -1.0, s1 = (B & 2) ? 1.0 : -1.0, s2 = (B & 4) ? 1.0 : -1.0;
  d[0] = s0 * a1 * a2;
  d[1] = a0 * s1 * a2;
  d[2] = a0 * a1 * s2;
  return a0 * a1 * a2;
}

// Bilinear factor of the vertex functions with bit s along D on the face
// xi_D = s: the product of the tangential factors at (t1, t2) for the vertex
// with tangential bits (j & 1, j >> 1).
__device__ __forceinline__ double vtx_face(int j, double t1, double t2) {
  return ((j & 1) ? t1 : 1.0 - t1) * ((j & 2) ? t2 : 1.0 - t2);
}
// Vertex index B of the vertex with bit s along D and tangential bits j.
template <int D>
__device__ __forceinline__ int vtx_index(int s, int j) {
  constexpr int T1 = D == 0 ? 1 : 0, T2 = D == 2 ? 1 : 2;
  return (s << D) | ((j & 1) << T1) | (((j >> 1) & 1) << T2);
}

// The tables of both bases at both rules are compile-time literals (ct::).
template <int NP, int NQ>
using MS = ct::MatS<NP, NQ>;
template <int NP, int NQ>
using MD = ct::MatSd<NP, NQ>;

// ---------------------------------------------------------------------------
// Velocity divergence: out = C u (pressure layout).

// Faces of direction D: {{u_D}} n_D at the face points (u_D- on walls), integrated against
// the pressure face layer, accumulated into acc.
template <int NPU, int NPP, int NQ, int NQY, bool ENR, int LE, int D>
__device__ __forceinline__ void div_faces(const DgArgs& A, const CellGeo& g, const double* su, const double* nl,
                                          const double* ut, const double* utn, const int64_t* nbf,
                                          const int64_t* nbe, double* w0, double* w1, double* acc, int tid) {
  constexpr int NU3 = NPU * NPU * NPU, NU2 = NPU * NPU;
  constexpr int T1 = D == 0 ? 1 : 0, T2 = D == 2 ? 1 : 2;
  constexpr int Q1 = T1 == 1 ? NQY : NQ, Q2 = T2 == 1 ? NQY : NQ;
  constexpr auto& tb1 = ct::tab<NPU, Q1>;
  constexpr auto& tb2 = ct::tab<NPU, Q2>;
  // layers of component D: [s][side][l1 + NPU l2] (side 0 own, 1 neighbour)
  for (int it = tid; it < 4 * NU2; it += kDgThreads) {
    const int r = it / NU2, l = it - r * NU2, s = r >> 1;
    w0[it] = (r & 1) ? nl[(2 * D + s) * NU2 + l] : su[D * NU3 + layer_node<NPU>(D, s, l % NPU, l / NPU)];
  }
  __syncthreads();
  sweep_c<0, NPU, NPU, 1, Q1, false, false, MS<NPU, Q1>>(w0, NU2, w1, Q1 * NPU, 1.0, 4);
  __syncthreads();
  sweep_c<1, Q1, NPU, 1, Q2, false, false, MS<NPU, Q2>>(w1, Q1 * NPU, w0, Q1 * Q2, 1.0, 4);
  __syncthreads();
  const double area = g.h[T1] * g.h[T2];
  for (int it = tid; it < 2 * Q1 * Q2; it += kDgThreads) {
    const int s = it / (Q1 * Q2), pt = it - s * Q1 * Q2;
    const int q1 = pt % Q1, q2 = pt / Q1;
    // weights of the enrichment on this face: l = 0 the coefficient, l = 1 the
    // coefficients of the four vertices on the face times their bilinear factors
    double lo = 0.0, ln = 0.0;
    if (LE == 1) {
      lo = ENR ? ut[D] : 0.0;
      ln = utn[2 * D + s];
    } else {
      const double t1 = tb1.g[q1], t2 = tb2.g[q2];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const double f = vtx_face(j, t1, t2);
        if (ENR) lo += f * ut[D * LE + vtx_index<D>(s, j)];
        ln += f * utn[(2 * D + s) * 4 + j];
      }
    }
    double um = w0[(s * 2) * Q1 * Q2 + pt], up = um;  // interior value on a no-slip wall
    if (ENR) um += A.psi[(g.enr * A.psi_pts + A.psi_off[1 + 2 * D + s] + pt) * 4] * lo;
    if (nbf[2 * D + s] >= 0) {
      up = w0[(s * 2 + 1) * Q1 * Q2 + pt];
      const int64_t ne = nbe[2 * D + s];
      if (ne >= 0) up += A.psi[(ne * A.psi_pts + A.psi_off[1 + 2 * D + (1 - s)] + pt) * 4] * ln;
    } else {
      up = um;
    }
    w1[it] = tb1.w[q1] * tb2.w[q2] * area * (s ? 0.5 : -0.5) * (um + up);
  }
  __syncthreads();
  sweep_c<0, Q1, Q2, 1, NPP, true, false, MS<NPP, Q1>>(w1, Q1 * Q2, w0, NPP * Q2, 1.0, 2);
  __syncthreads();
  sweep_c<1, NPP, Q2, 1, NPP, true, false, MS<NPP, Q2>>(w0, NPP * Q2, w1, NPP * NPP, 1.0, 2);
  __syncthreads();
  // the two layers of direction D are disjoint (NPP >= 2)
  for (int it = tid; it < 2 * NPP * NPP; it += kDgThreads) {
    const int s = it / (NPP * NPP), l = it - s * NPP * NPP;
    acc[layer_node<NPP>(D, s, l % NPP, l / NPP)] += w1[it];
  }
  __syncthreads();
}

template <int NPU, int NPP, int NQ, int NQY, bool ENR, int LE>
__global__ __launch_bounds__(kDgThreads) void divergence_kernel(const DgArgs A, int layer_lo, int nlayers) {
  constexpr int NU3 = NPU * NPU * NPU, NP3 = NPP * NPP * NPP, NPT = NQ * NQY * NQ, NU2 = NPU * NPU;
  constexpr auto& tq = ct::tab<NPU, NQ>;
  constexpr auto& ty = ct::tab<NPU, NQY>;
  __shared__ double su[3 * NU3];
  __shared__ double w0[3 * NPT], w1[3 * NPT];    // work arrays (>= every intermediate)
  __shared__ double acc[NP3];
  __shared__ double nl[6 * NU2];                 // neighbours' normal-component layers at the shared faces
  __shared__ double ut[3 * LE];                  // u~ of the cell, [c][B]
  // normal u~ of each face's enriched neighbour (else 0); l = 1: its four
  // coefficients on the shared face, by tangential bits
  __shared__ double utn[LE == 1 ? 6 : 24];
  const int tid = threadIdx.x;
  const CellGeo g = cell_of_block<ENR>(A, blockIdx.x, layer_lo, nlayers);
  const int64_t e = g.e;
  int64_t nbf[6], nbe[6];
#pragma unroll
  for (int f = 0; f < 6; ++f) {
    int a, b, c;
    nbf[f] = neighbour(A, g, f >> 1, f & 1, a, b, c);
    nbe[f] = nbf[f] < 0 ? -1 : enr_of(A, a, b, c);
  }
  // every global read of the cell is issued before the first barrier
  const double* ue = A.in + e * 3 * NU3;
  for (int i = tid; i < 3 * NU3; i += kDgThreads) su[i] = ue[i];
  for (int it = tid; it < 6 * NU2; it += kDgThreads) {
    const int f = it / NU2, l = it - f * NU2, d = f >> 1, s = f & 1;
    nl[it] = nbf[f] < 0 ? 0.0 : A.in[(nbf[f] * 3 + d) * NU3 + layer_node<NPU>(d, 1 - s, l % NPU, l / NPU)];
  }
  if (ENR && tid < 3 * LE) ut[tid] = A.in[A.ncell * 3 * NU3 + g.enr * 3 * LE + tid];
  if (LE == 1) {
    if (tid >= 64 && tid < 70) {
      const int f = tid - 64;
      utn[f] = nbe[f] >= 0 ? A.in[A.ncell * 3 * NU3 + nbe[f] * 3 + (f >> 1)] : 0.0;
    }
  } else if (tid >= 64 && tid < 88) {
    // the neighbour across face (d, s) meets it at its own xi_d = 1 - s
    const int f = (tid - 64) >> 2, j = (tid - 64) & 3, d = f >> 1, sn = 1 - (f & 1);
    const int B = d == 0 ? vtx_index<0>(sn, j) : (d == 1 ? vtx_index<1>(sn, j) : vtx_index<2>(sn, j));
    utn[tid - 64] = nbe[f] >= 0 ? A.in[A.ncell * 3 * NU3 + nbe[f] * 3 * LE + d * LE + B] : 0.0;
  }
  __syncthreads();
  const double detJ = g.h[0] * g.h[1] * g.h[2];
  // ---- volume: u at the points, f_c = -w |J| u_c / h_c, c = sum_c (d_c N^p)^T f_c
  sweep_c<0, NPU, NPU, NPU, NQ, false, false, MS<NPU, NQ>>(su, NU3, w0, NPT, 1.0, 3);
  __syncthreads();
  sweep_c<1, NQ, NPU, NPU, NQY, false, false, MS<NPU, NQY>>(w0, NPT, w1, NPT, 1.0, 3);
  __syncthreads();
  sweep_c<2, NQ, NQY, NPU, NQ, false, false, MS<NPU, NQ>>(w1, NPT, w0, NPT, 1.0, 3);
  __syncthreads();
  for (int it = tid; it < 3 * NPT; it += kDgThreads) {
    const int c = it / NPT, q = it - c * NPT;
    const int qx = q % NQ, qy = (q / NQ) % NQY, qz = q / (NQ * NQY);
    double v = w0[it];
    if (ENR) {
      double L = ut[c * LE];
      if (LE == 8) {
        const double x[3] = {tq.g[qx], ty.g[qy], tq.g[qz]};
        double dd[3];
        L = 0.0;
#pragma unroll
        for (int B = 0; B < 8; ++B) L += vtx(B, x, dd) * ut[c * LE + B];
      }
      v += A.psi[(g.enr * A.psi_pts + q) * 4] * L;
    }
    w0[it] = -tq.w[qx] * ty.w[qy] * tq.w[qz] * detJ / g.h[c] * v;
  }
  __syncthreads();
  // component c is tested with d_c N^p; the three sweeps of a phase use separate wavefronts
  sweep_c<0, NQ, NQY, NQ, NPP, true, false, MD<NPP, NQ>>(w0, NPT, w1, NPT, 1.0, 1, 0);
  sweep_c<0, NQ, NQY, NQ, NPP, true, false, MS<NPP, NQ>>(w0 + NPT, NPT, w1 + NPT, NPT, 1.0, 1, 64);
  sweep_c<0, NQ, NQY, NQ, NPP, true, false, MS<NPP, NQ>>(w0 + 2 * NPT, NPT, w1 + 2 * NPT, NPT, 1.0, 1, 128);
  __syncthreads();
  sweep_c<1, NPP, NQY, NQ, NPP, true, false, MS<NPP, NQY>>(w1, NPT, w0, NPT, 1.0, 1, 0);
  sweep_c<1, NPP, NQY, NQ, NPP, true, false, MD<NPP, NQY>>(w1 + NPT, NPT, w0 + NPT, NPT, 1.0, 1, 64);
  sweep_c<1, NPP, NQY, NQ, NPP, true, false, MS<NPP, NQY>>(w1 + 2 * NPT, NPT, w0 + 2 * NPT, NPT, 1.0, 1, 128);
  __syncthreads();
  sweep_c<2, NPP, NPP, NQ, NPP, true, false, MS<NPP, NQ>>(w0, NPT, w1, NPT, 1.0, 1, 0);
  sweep_c<2, NPP, NPP, NQ, NPP, true, false, MS<NPP, NQ>>(w0 + NPT, NPT, w1 + NPT, NPT, 1.0, 1, 64);
  sweep_c<2, NPP, NPP, NQ, NPP, true, false, MD<NPP, NQ>>(w0 + 2 * NPT, NPT, w1 + 2 * NPT, NPT, 1.0, 1, 128);
  __syncthreads();
  for (int B = tid; B < NP3; B += kDgThreads) acc[B] = w1[B] + w1[NPT + B] + w1[2 * NPT + B];
  __syncthreads();
  // ---- faces, direction by direction
  div_faces<NPU, NPP, NQ, NQY, ENR, LE, 0>(A, g, su, nl, ut, utn, nbf, nbe, w0, w1, acc, tid);
  div_faces<NPU, NPP, NQ, NQY, ENR, LE, 1>(A, g, su, nl, ut, utn, nbf, nbe, w0, w1, acc, tid);
  div_faces<NPU, NPP, NQ, NQY, ENR, LE, 2>(A, g, su, nl, ut, utn, nbf, nbe, w0, w1, acc, tid);
  double* oe = A.out + e * NP3;
  for (int B = tid; B < NP3; B += kDgThreads) oe[B] = acc[B];
}

// ---------------------------------------------------------------------------
// Pressure gradient: out = P p (velocity layout, enrichment rows included).

// Faces of direction D: n_D {{p}} at the face points, integrated against the
// velocity face layer of component D (and psi for the enrichment row D).
template <int NPU, int NPP, int NQ, int NQY, bool ENR, int LE, int D>
__device__ __forceinline__ void grad_faces(const DgArgs& A, const CellGeo& g, const double* sp, const double* nl,
                                           const int64_t* nbf, double* w0, double* w1, double* acc, double* red,
                                           double* accE, int tid) {
  constexpr int NU3 = NPU * NPU * NPU, NP2 = NPP * NPP;
  constexpr int T1 = D == 0 ? 1 : 0, T2 = D == 2 ? 1 : 2;
  constexpr int Q1 = T1 == 1 ? NQY : NQ, Q2 = T2 == 1 ? NQY : NQ;
  constexpr auto& tb1 = ct::tab<NPU, Q1>;
  constexpr auto& tb2 = ct::tab<NPU, Q2>;
  constexpr int NW = kDgThreads / 64;
  // pressure layers [s][side][l1 + NPP l2]; a wall repeats the own layer (p+ = p-)
  for (int it = tid; it < 4 * NP2; it += kDgThreads) {
    const int r = it / NP2, l = it - r * NP2, s = r >> 1;
    w0[it] = ((r & 1) && nbf[2 * D + s] >= 0) ? nl[(2 * D + s) * NP2 + l]
                                               : sp[layer_node<NPP>(D, s, l % NPP, l / NPP)];
  }
  __syncthreads();
  sweep_c<0, NPP, NPP, 1, Q1, false, false, MS<NPP, Q1>>(w0, NP2, w1, Q1 * NPP, 1.0, 4);
  __syncthreads();
  sweep_c<1, Q1, NPP, 1, Q2, false, false, MS<NPP, Q2>>(w1, Q1 * NPP, w0, Q1 * Q2, 1.0, 4);
  __syncthreads();
  const double area = g.h[T1] * g.h[T2];
  // enrichment rows of component D: l = 0 one sum; l = 1 the four vertices on
  // each of the two faces (the others vanish there), [s][tangential bits]
  constexpr int NE = LE == 1 ? 1 : 8;
  double ve[NE];
#pragma unroll
  for (int i = 0; i < NE; ++i) ve[i] = 0.0;
  for (int it = tid; it < 2 * Q1 * Q2; it += kDgThreads) {
    const int s = it / (Q1 * Q2), pt = it - s * Q1 * Q2;
    const int q1 = pt % Q1, q2 = pt / Q1;
    const double fl = tb1.w[q1] * tb2.w[q2] * area * (s ? 0.5 : -0.5) *
                      (w0[(s * 2) * Q1 * Q2 + pt] + w0[(s * 2 + 1) * Q1 * Q2 + pt]);
    w1[it] = fl;
    if (ENR) {
      const double pf = A.psi[(g.enr * A.psi_pts + A.psi_off[1 + 2 * D + s] + pt) * 4] * fl;
      if (LE == 1) {
        ve[0] += pf;
      } else {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const double f = vtx_face(j, tb1.g[q1], tb2.g[q2]) * pf;
          ve[j] += s ? 0.0 : f;
          ve[4 + j] += s ? f : 0.0;
        }
      }
    }
  }
  if (ENR) {
    block_sum_n<NE>(ve, red);  // (its barrier also publishes w1)
    if (tid < NE) {
      if (LE == 1) accE[D] += ve[0];
      else accE[D * LE + vtx_index<D>(tid >> 2, tid & 3)] += ve[0];
    }
  } else {
    __syncthreads();
  }
  sweep_c<0, Q1, Q2, 1, NPU, true, false, MS<NPU, Q1>>(w1, Q1 * Q2, w0, NPU * Q2, 1.0, 2);
  __syncthreads();
  sweep_c<1, NPU, Q2, 1, NPU, true, false, MS<NPU, Q2>>(w0, NPU * Q2, w1, NPU * NPU, 1.0, 2);
  __syncthreads();
  for (int it = tid; it < 2 * NPU * NPU; it += kDgThreads) {
    const int s = it / (NPU * NPU), l = it - s * NPU * NPU;
    acc[D * NU3 + layer_node<NPU>(D, s, l % NPU, l / NPU)] += w1[it];
  }
  __syncthreads();
}

template <int NPU, int NPP, int NQ, int NQY, bool ENR, int LE>
__global__ __launch_bounds__(kDgThreads) void gradient_kernel(const DgArgs A, int layer_lo, int nlayers) {
  constexpr int NU3 = NPU * NPU * NPU, NP3 = NPP * NPP * NPP, NPT = NQ * NQY * NQ, NP2 = NPP * NPP;
  constexpr auto& tq = ct::tab<NPU, NQ>;
  constexpr auto& ty = ct::tab<NPU, NQY>;
  constexpr int NW = kDgThreads / 64;
  __shared__ double sp[NP3];
  __shared__ double w0[3 * NPT], w1[3 * NPT];
  __shared__ double acc[3 * NU3];
  __shared__ double nl[6 * NP2];                 // neighbours' pressure layers at the shared faces
  __shared__ double red[3 * LE * NW];
  __shared__ double accE[3 * LE];                // enrichment rows [c][B]
  const int tid = threadIdx.x;
  const CellGeo g = cell_of_block<ENR>(A, blockIdx.x, layer_lo, nlayers);
  const int64_t e = g.e;
  int64_t nbf[6];
#pragma unroll
  for (int f = 0; f < 6; ++f) {
    int a, b, c;
    nbf[f] = neighbour(A, g, f >> 1, f & 1, a, b, c);
  }
  const double* pe = A.in + e * NP3;
  for (int i = tid; i < NP3; i += kDgThreads) sp[i] = pe[i];
  for (int it = tid; it < 6 * NP2; it += kDgThreads) {
    const int f = it / NP2, l = it - f * NP2, d = f >> 1, s = f & 1;
    nl[it] = nbf[f] < 0 ? 0.0 : A.in[nbf[f] * NP3 + layer_node<NPP>(d, 1 - s, l % NPP, l / NPP)];
  }
  __syncthreads();
  const double detJ = g.h[0] * g.h[1] * g.h[2];
  // ---- volume: p at the points, g_c = -(d_c N^u)^T (w |J| p) / h_c
  sweep_c<0, NPP, NPP, NPP, NQ, false, false, MS<NPP, NQ>>(sp, NP3, w0, NPT, 1.0, 1);
  __syncthreads();
  sweep_c<1, NQ, NPP, NPP, NQY, false, false, MS<NPP, NQY>>(w0, NPT, w1, NPT, 1.0, 1);
  __syncthreads();
  sweep_c<2, NQ, NQY, NPP, NQ, false, false, MS<NPP, NQ>>(w1, NPT, w0, NPT, 1.0, 1);
  __syncthreads();
  // enrichment rows: -(div(phi e_c), p) with phi = psi (l = 0) or psi N_B (l = 1),
  // d_c phi = N_B d_c psi + psi d_c N_B
  double ve[3 * LE];
#pragma unroll
  for (int i = 0; i < 3 * LE; ++i) ve[i] = 0.0;
  for (int q = tid; q < NPT; q += kDgThreads) {
    const int qx = q % NQ, qy = (q / NQ) % NQY, qz = q / (NQ * NQY);
    const double v = -tq.w[qx] * ty.w[qy] * tq.w[qz] * detJ * w0[q];
    if (ENR) {
      const double* ps = A.psi + (g.enr * A.psi_pts + q) * 4;
      if (LE == 1) {
        ve[0] += ps[1] * v;
        ve[1] += ps[2] * v;
        ve[2] += ps[3] * v;
      } else {
        const double x[3] = {tq.g[qx], ty.g[qy], tq.g[qz]};
#pragma unroll
        for (int B = 0; B < LE; ++B) {
          double dd[3];
          const double nb = vtx(B, x, dd);
#pragma unroll
          for (int c = 0; c < 3; ++c) ve[c * LE + B] += (nb * ps[1 + c] + ps[0] * dd[c] / g.h[c]) * v;
        }
      }
    }
    w1[q] = v / g.h[0];
    w1[NPT + q] = v / g.h[1];
    w1[2 * NPT + q] = v / g.h[2];
  }
  if (ENR) {
    block_sum_n<3 * LE>(ve, red);  // (its barrier also publishes w1)
    if (tid < 3 * LE) accE[tid] = ve[0];
  } else {
    __syncthreads();
  }
  // component c tested with d_c N^u; the three sweeps of a phase use separate wavefronts
  sweep_c<0, NQ, NQY, NQ, NPU, true, false, MD<NPU, NQ>>(w1, NPT, w0, NPT, 1.0, 1, 0);
  sweep_c<0, NQ, NQY, NQ, NPU, true, false, MS<NPU, NQ>>(w1 + NPT, NPT, w0 + NPT, NPT, 1.0, 1, 64);
  sweep_c<0, NQ, NQY, NQ, NPU, true, false, MS<NPU, NQ>>(w1 + 2 * NPT, NPT, w0 + 2 * NPT, NPT, 1.0, 1, 128);
  __syncthreads();
  sweep_c<1, NPU, NQY, NQ, NPU, true, false, MS<NPU, NQY>>(w0, NPT, w1, NPT, 1.0, 1, 0);
  sweep_c<1, NPU, NQY, NQ, NPU, true, false, MD<NPU, NQY>>(w0 + NPT, NPT, w1 + NPT, NPT, 1.0, 1, 64);
  sweep_c<1, NPU, NQY, NQ, NPU, true, false, MS<NPU, NQY>>(w0 + 2 * NPT, NPT, w1 + 2 * NPT, NPT, 1.0, 1, 128);
  __syncthreads();
  sweep_c<2, NPU, NPU, NQ, NPU, true, false, MS<NPU, NQ>>(w1, NPT, acc, NU3, 1.0, 1, 0);
  sweep_c<2, NPU, NPU, NQ, NPU, true, false, MS<NPU, NQ>>(w1 + NPT, NPT, acc + NU3, NU3, 1.0, 1, 64);
  sweep_c<2, NPU, NPU, NQ, NPU, true, false, MD<NPU, NQ>>(w1 + 2 * NPT, NPT, acc + 2 * NU3, NU3, 1.0, 1, 128);
  __syncthreads();
  // ---- faces
  grad_faces<NPU, NPP, NQ, NQY, ENR, LE, 0>(A, g, sp, nl, nbf, w0, w1, acc, red, accE, tid);
  grad_faces<NPU, NPP, NQ, NQY, ENR, LE, 1>(A, g, sp, nl, nbf, w0, w1, acc, red, accE, tid);
  grad_faces<NPU, NPP, NQ, NQY, ENR, LE, 2>(A, g, sp, nl, nbf, w0, w1, acc, red, accE, tid);
  double* oe = A.out + e * 3 * NU3;
  for (int B = tid; B < 3 * NU3; B += kDgThreads) oe[B] = acc[B];
  if (ENR && tid < 3 * LE) A.out[A.ncell * 3 * NU3 + g.enr * 3 * LE + tid] = accE[tid];
}

}  // namespace

// (k_u+1, k_p+1, nq_u, nq_wn) combinations: the velocity ones with k_p = k_u - 1
#define DG_DG_COMBOS(X) X(3, 2, 4, 8) X(3, 2, 4, 4) X(4, 3, 4, 8) X(4, 3, 5, 8) X(4, 3, 5, 5) X(5, 4, 7, 8) X(6, 5, 8, 8)

int launch_divgrad(const dg_mesh* m, bool divergence, const double* in, double* out, hipStream_t s) {
  if (m->curved) return launch_divgrad_curved(m, divergence, in, out, s);
  DgArgs A;
  A.nx = m->P.nx;
  A.ny = m->P.ny;
  A.nz = m->P.nz;
  A.lower_slot = m->lower_slot;
  A.upper_slot = m->upper_slot;
  A.nslots = m->n_enr_layers;
  A.psi_pts = m->psi_pts;
  A.fully_periodic = m->P.fully_periodic;
  A.psi_off[0] = 0;
  for (int f = 0; f < 6; ++f) A.psi_off[1 + f] = psi_face_offset(m->P.nq_u, m->P.nq_wn, f);
  A.ncell = m->ncell;
  A.hx = m->hx;
  A.hz = m->hz;
  A.hy = m->hy;
  A.psi = m->psi;
  A.in = in;
  A.out = out;
  const int lo = (m->P.fully_periodic || m->lower_slot < 0) ? 0 : 1;
  const int hi = (m->P.fully_periodic || m->upper_slot < 0) ? m->P.ny - 1 : m->P.ny - 2;
  const int nl = hi - lo + 1;
  const int64_t nreg = nl > 0 ? (int64_t)m->P.nx * nl * m->P.nz : 0;
  // without enriched cells only the regular kernels run and nq_wn is irrelevant
  const bool any_w = m->nenr == 0;
  const int nqw = m->P.nq_wn;
#define LAUNCH(KER, pu, pp, q, w, ENRV, LEV, grid, lo_, nl_)                                            \
  hipLaunchKernelGGL((KER<pu, pp, q, w, ENRV, LEV>), dim3((unsigned)(grid)), dim3(kDgThreads), 0, s, A, lo_, nl_)
#define RUN(LEV, pu, pp, q, w)                                                                           \
  {                                                                                                      \
    if (nreg > 0) {                                                                                      \
      if (divergence) LAUNCH(divergence_kernel, pu, pp, q, q, false, LEV, nreg, lo, nl);                  \
      else LAUNCH(gradient_kernel, pu, pp, q, q, false, LEV, nreg, lo, nl);                               \
      const int rc = check_hip(hipGetLastError(), "divergence/gradient kernel launch");                  \
      if (rc) return rc;                                                                                 \
    }                                                                                                    \
    if (m->nenr > 0) {                                                                                   \
      if (divergence) LAUNCH(divergence_kernel, pu, pp, q, w, true, LEV, m->nenr, 0, 0);                  \
      else LAUNCH(gradient_kernel, pu, pp, q, w, true, LEV, m->nenr, 0, 0);                               \
    }                                                                                                    \
    return check_hip(hipGetLastError(), "divergence/gradient kernel launch");                            \
  }
#define X(pu, pp, q, w)                                                                                  \
  if (m->np_u == pu && m->np_p == pp && m->P.nq_u == q && (any_w || nqw == w)) {                          \
    if (m->nle == 8) RUN(8, pu, pp, q, w)                                                                \
    else RUN(1, pu, pp, q, w)                                                                            \
  }
  DG_DG_COMBOS(X)
#undef X
#undef RUN
#undef LAUNCH
  return set_error(DG_ERR_UNSUPPORTED,
                   "pressure gradient / velocity divergence: (k_u+1, k_p+1, nq_u, nq_wn) combination not compiled");
}

}  // namespace dgwm
