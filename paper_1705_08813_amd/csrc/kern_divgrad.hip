// Pressure gradient and velocity divergence terms of the dual-splitting
// scheme (arXiv 1705.08813, Sec. 4.2), FP64, flat (box) meshes.
//
//   P: g(v) = -(div v, p)_e + (v . n, {{p}})_{boundary of e}     (velocity test functions)
//   C: c(q) = -(grad q, u)_e + (q, {{u}} . n)_{boundary of e}    (pressure test functions)
//
// {{.}} the central average; on no-slip walls the external values are
// p+ = p- and u+ = -u- (so {{u}} = 0 there).  u is the full velocity with
// psi u~ in enriched cells, and the velocity test functions include psi e_c.
// Both use the velocity quadrature of the cell (nq^3, nq x nqy x nq in
// enriched cells) and of its faces (x- and z-faces take the cell's
// wall-normal rule, which every neighbour in the same layer shares).
//
// One workgroup per cell; the output block of the cell is accumulated in LDS
// (volume term first, then the faces direction by direction) and written
// once, so every output has one writer.  Values at points come from
// sum-factorized interpolation sweeps, test-function integrals from the
// transposed sweeps; faces interpolate the node layer at the face (the
// Gauss-Lobatto nodal basis has its face values on that layer) of the cell
// and of its neighbour.  The pressure basis is tabulated at the velocity
// rule's points (a table of its own, same layout as the velocity tables).
#include "kern_common.h"

namespace dgwm {

namespace {

constexpr int kDgThreads = 256;

// out[c][...] = sum_l A_c[o][l] in[c][...] along direction DIR of NC stacked
// 3-D arrays with strides (1, E0, E0 E1); E = extents of `in`, MO = output
// extent along DIR; A_c is [MO][L] (TR: [L][MO], i.e. A_c^T is applied),
// A_0, A_1, A_2 for components 0, 1, 2.
template <int NC, int DIR, int E0, int E1, int E2, int MO, bool TR>
__device__ __forceinline__ void sweepm(const double* in, double* out, const double* A0, const double* A1,
                                       const double* A2, int tid) {
  constexpr int L = DIR == 0 ? E0 : DIR == 1 ? E1 : E2;
  constexpr int O0 = DIR == 0 ? MO : E0, O1 = DIR == 1 ? MO : E1, O2 = DIR == 2 ? MO : E2;
  constexpr int NI = E0 * E1 * E2, NO = O0 * O1 * O2;
  constexpr int st = DIR == 0 ? 1 : DIR == 1 ? E0 : E0 * E1;
  for (int it = tid; it < NC * NO; it += kDgThreads) {
    const int c = it / NO, r = it - c * NO;
    const int o0 = r % O0, o1 = (r / O0) % O1, o2 = r / (O0 * O1);
    const int o = DIR == 0 ? o0 : DIR == 1 ? o1 : o2;
    const int base = (DIR == 0 ? 0 : o0) + E0 * ((DIR == 1 ? 0 : o1) + E1 * (DIR == 2 ? 0 : o2));
    const double* ip = in + c * NI + base;
    const double* a = c == 0 ? A0 : (c == 1 ? A1 : A2);
    double s = 0.0;
#pragma unroll
    for (int l = 0; l < L; ++l) s += (TR ? a[l * MO + o] : a[o * L + l]) * ip[l * st];
    out[it] = s;
  }
}

struct DgArgs {
  int nx, ny, nz, lower_slot, upper_slot, nslots, psi_pts, fully_periodic;
  int psi_off[7];          // volume, then the six faces f = 2d + s
  int64_t ncell;
  double hx, hz;
  const double* hy;        // ny heights
  const double* tab_u;     // velocity basis tables at the velocity rules
  const double* tab_pu;    // pressure basis tables at the velocity rules
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

__device__ __forceinline__ CellGeo cell_geo(const DgArgs& A, int64_t e) {
  CellGeo g;
  g.e = e;
  g.ex = (int)(e % A.nx);
  const int64_t t = e / A.nx;
  g.ey = (int)(t % A.ny);
  g.ez = (int)(t / A.ny);
  g.enr = enr_of(A, g.ex, g.ey, g.ez);
  g.h[0] = A.hx;
  g.h[1] = A.hy[g.ey];
  g.h[2] = A.hz;
  return g;
}

// Neighbour across face (d, s): cell index, or -1 on a no-slip wall.
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

// Node index (i, j, k along x, y, z) of position (l1, l2) on the layer of face
// (d, s) of an NP^3 nodal block: tangential directions t1 < t2.
template <int NP>
__device__ __forceinline__ int layer_node(int d, int s, int l1, int l2) {
  const int ld = s ? NP - 1 : 0;
  if (d == 0) return ld + NP * (l1 + NP * l2);
  if (d == 1) return l1 + NP * (ld + NP * l2);
  return l1 + NP * (l2 + NP * ld);
}

// 1-D tables of both bases, in LDS: the wall-parallel rule and the rule
// along y (the wall-normal rule in enriched cells, the same rule otherwise).
template <int NPU, int NPP, int NQ, int NQY>
struct DgTab {
  double Su[NQ * NPU], Du[NQ * NPU], Suy[NQY * NPU], Duy[NQY * NPU];
  double Sp[NQ * NPP], Dp[NQ * NPP], Spy[NQY * NPP], Dpy[NQY * NPP];
  double W[NQ], Wy[NQY];
};

template <int NPU, int NPP, int NQ, int NQY, bool ENR>
__device__ __forceinline__ void load_dgtab(const DgArgs& A, DgTab<NPU, NPP, NQ, NQY>& T, int tid) {
  // the tables were built for (np, nq_u, nq_wn); offsets before the y rule depend on (np, nq) only
  constexpr TabLayout Lu = tab_layout(NPU, NQ, NQY), Lp = tab_layout(NPP, NQ, NQY);
  static_assert(ENR || NQY == NQ, "regular cells use one rule");
  constexpr int uSy = ENR ? Lu.Sy : Lu.S, uSdy = ENR ? Lu.Sdy : Lu.Sd, uwy = ENR ? Lu.wy : Lu.w;
  constexpr int pSy = ENR ? Lp.Sy : Lp.S, pSdy = ENR ? Lp.Sdy : Lp.Sd;
  for (int i = tid; i < NQ * NPU; i += kDgThreads) {
    T.Su[i] = A.tab_u[Lu.S + i];
    T.Du[i] = A.tab_u[Lu.Sd + i];
  }
  for (int i = tid; i < NQY * NPU; i += kDgThreads) {
    T.Suy[i] = A.tab_u[uSy + i];
    T.Duy[i] = A.tab_u[uSdy + i];
  }
  for (int i = tid; i < NQ * NPP; i += kDgThreads) {
    T.Sp[i] = A.tab_pu[Lp.S + i];
    T.Dp[i] = A.tab_pu[Lp.Sd + i];
  }
  for (int i = tid; i < NQY * NPP; i += kDgThreads) {
    T.Spy[i] = A.tab_pu[pSy + i];
    T.Dpy[i] = A.tab_pu[pSdy + i];
  }
  if (tid < NQ) T.W[tid] = A.tab_u[Lu.w + tid];
  if (tid < NQY) T.Wy[tid] = A.tab_u[uwy + tid];
}

// ---------------------------------------------------------------------------
// Velocity divergence: out = C u (pressure layout).
template <int NPU, int NPP, int NQ, int NQY, bool ENR>
__global__ __launch_bounds__(kDgThreads) void divergence_kernel(const DgArgs A, int layer_lo, int nlayers) {
  constexpr int NU3 = NPU * NPU * NPU, NP3 = NPP * NPP * NPP, NPT = NQ * NQY * NQ;
  __shared__ DgTab<NPU, NPP, NQ, NQY> T;
  __shared__ double su[3 * NU3];
  __shared__ double w0[3 * NPT], w1[3 * NPT];    // work arrays (>= every intermediate)
  __shared__ double acc[NP3];
  __shared__ double ut[2][3];                     // u~ of the cell and (per face) of the neighbour
  const int tid = threadIdx.x;
  int64_t e;
  if (ENR) {
    const int64_t b = blockIdx.x;
    const int ex = (int)(b % A.nx);
    const int64_t t0 = b / A.nx;
    const int slot = (int)(t0 % A.nslots);
    const int ez = (int)(t0 / A.nslots);
    const int ey = slot == A.lower_slot ? 0 : A.ny - 1;
    e = ex + (int64_t)A.nx * (ey + (int64_t)A.ny * ez);
  } else {
    const int64_t b = blockIdx.x;
    const int ex = (int)(b % A.nx);
    const int64_t t0 = b / A.nx;
    e = ex + (int64_t)A.nx * (layer_lo + (int)(t0 % nlayers) + (int64_t)A.ny * (t0 / nlayers));
  }
  const CellGeo g = cell_geo(A, e);
  load_dgtab<NPU, NPP, NQ, NQY, ENR>(A, T, tid);
  const double* ue = A.in + e * 3 * NU3;
  for (int i = tid; i < 3 * NU3; i += kDgThreads) su[i] = ue[i];
  if (ENR && tid < 3) ut[0][tid] = A.in[A.ncell * 3 * NU3 + g.enr * 3 + tid];
  __syncthreads();
  const double detJ = g.h[0] * g.h[1] * g.h[2];
  // ---- volume: u at the points, f_d = w |J| u_d / h_d, c = -sum_d (d_d N^p)^T f_d
  {
    sweepm<3, 0, NPU, NPU, NPU, NQ, false>(su, w0, T.Su, T.Su, T.Su, tid);       // [c][k][j][qx]
    __syncthreads();
    sweepm<3, 1, NQ, NPU, NPU, NQY, false>(w0, w1, T.Suy, T.Suy, T.Suy, tid);   // [c][k][qy][qx]
    __syncthreads();
    sweepm<3, 2, NQ, NQY, NPU, NQ, false>(w1, w0, T.Su, T.Su, T.Su, tid);       // [c][qz][qy][qx]
    __syncthreads();
    for (int it = tid; it < 3 * NPT; it += kDgThreads) {
      const int c = it / NPT, q = it - c * NPT;
      const int qx = q % NQ, qy = (q / NQ) % NQY, qz = q / (NQ * NQY);
      double v = w0[it];
      if (ENR) v += A.psi[(g.enr * A.psi_pts + q) * 4] * ut[0][c];
      w0[it] = -T.W[qx] * T.Wy[qy] * T.W[qz] * detJ / g.h[c] * v;
    }
    __syncthreads();
    // component d is tested with d_d N^p: derivative table along d, values elsewhere
    sweepm<3, 0, NQ, NQY, NQ, NPP, true>(w0, w1, T.Dp, T.Sp, T.Sp, tid);       // [c][qz][qy][i]
    __syncthreads();
    sweepm<3, 1, NPP, NQY, NQ, NPP, true>(w1, w0, T.Spy, T.Dpy, T.Spy, tid);   // [c][qz][j][i]
    __syncthreads();
    sweepm<3, 2, NPP, NPP, NQ, NPP, true>(w0, w1, T.Sp, T.Sp, T.Dp, tid);      // [c][k][j][i]
    __syncthreads();
    for (int B = tid; B < NP3; B += kDgThreads) acc[B] = w1[B] + w1[NP3 + B] + w1[2 * NP3 + B];
    __syncthreads();
  }
  // ---- faces, direction by direction: (q, {{u}} . n) on the pressure face layer
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
    const int Q1 = t1 == 1 ? NQY : NQ, Q2 = t2 == 1 ? NQY : NQ;
    int nbi[2][3];
    int64_t nb[2], nbe[2];
    for (int s = 0; s < 2; ++s) {
      nb[s] = neighbour(A, g, d, s, nbi[s][0], nbi[s][1], nbi[s][2]);
      nbe[s] = nb[s] < 0 ? -1 : enr_of(A, nbi[s][0], nbi[s][1], nbi[s][2]);
    }
    // layers of component d: [s][side][l1 + NPU l2] (side 0 own, 1 neighbour)
    for (int it = tid; it < 4 * NPU * NPU; it += kDgThreads) {
      const int r = it / (NPU * NPU), l = it - r * NPU * NPU;
      const int s = r >> 1, side = r & 1;
      const int l1 = l % NPU, l2 = l / NPU;
      double v = 0.0;
      if (side == 0) v = su[d * NU3 + layer_node<NPU>(d, s, l1, l2)];
      else if (nb[s] >= 0) v = A.in[(nb[s] * 3 + d) * NU3 + layer_node<NPU>(d, 1 - s, l1, l2)];
      w0[it] = v;
    }
    if (tid < 2) {
      const int s = tid;
      ut[1][s] = nbe[s] >= 0 ? A.in[A.ncell * 3 * NU3 + nbe[s] * 3 + d] : 0.0;
    }
    __syncthreads();
    // interpolate to the face points: [s][side][q1 + Q1 q2]
    const double* T1S = t1 == 1 ? T.Suy : T.Su;
    const double* T2S = t2 == 1 ? T.Suy : T.Su;
    for (int it = tid; it < 4 * Q1 * NPU; it += kDgThreads) {
      const int r = it / (Q1 * NPU), l = it - r * Q1 * NPU;
      const int q1 = l % Q1, l2 = l / Q1;
      const double* ip = w0 + r * NPU * NPU + NPU * l2;
      double s = 0.0;
      for (int l1 = 0; l1 < NPU; ++l1) s += T1S[q1 * NPU + l1] * ip[l1];
      w1[it] = s;
    }
    __syncthreads();
    for (int it = tid; it < 4 * Q1 * Q2; it += kDgThreads) {
      const int r = it / (Q1 * Q2), l = it - r * Q1 * Q2;
      const int q1 = l % Q1, q2 = l / Q1;
      const double* ip = w1 + r * Q1 * NPU + q1;
      double s = 0.0;
      for (int l2 = 0; l2 < NPU; ++l2) s += T2S[q2 * NPU + l2] * ip[l2 * Q1];
      w0[it] = s;
    }
    __syncthreads();
    // flux at each face point: w |F| n_d {{u_d}}, zero on walls
    const double area = g.h[t1] * g.h[t2];
    const double* W1 = t1 == 1 ? T.Wy : T.W;
    const double* W2 = t2 == 1 ? T.Wy : T.W;
    for (int it = tid; it < 2 * Q1 * Q2; it += kDgThreads) {
      const int s = it / (Q1 * Q2), pt = it - s * Q1 * Q2;
      const int q1 = pt % Q1, q2 = pt / Q1;
      double f = 0.0;
      if (nb[s] >= 0) {
        double um = w0[(s * 2 + 0) * Q1 * Q2 + pt], up = w0[(s * 2 + 1) * Q1 * Q2 + pt];
        if (ENR) um += A.psi[(g.enr * A.psi_pts + A.psi_off[1 + 2 * d + s] + pt) * 4] * ut[0][d];
        if (nbe[s] >= 0) up += A.psi[(nbe[s] * A.psi_pts + A.psi_off[1 + 2 * d + (1 - s)] + pt) * 4] * ut[1][s];
        f = W1[q1] * W2[q2] * area * (s ? 0.5 : -0.5) * (um + up);
      }
      w1[it] = f;
    }
    __syncthreads();
    // integrate against the pressure face layer: [s][l1 + NPP l2]
    const double* P1 = t1 == 1 ? T.Spy : T.Sp;
    const double* P2 = t2 == 1 ? T.Spy : T.Sp;
    for (int it = tid; it < 2 * NPP * Q2; it += kDgThreads) {
      const int s = it / (NPP * Q2), l = it - s * NPP * Q2;
      const int l1 = l % NPP, q2 = l / NPP;
      const double* ip = w1 + s * Q1 * Q2 + Q1 * q2;
      double v = 0.0;
      for (int q1 = 0; q1 < Q1; ++q1) v += P1[q1 * NPP + l1] * ip[q1];
      w0[it] = v;
    }
    __syncthreads();
    for (int it = tid; it < 2 * NPP * NPP; it += kDgThreads) {
      const int s = it / (NPP * NPP), l = it - s * NPP * NPP;
      const int l1 = l % NPP, l2 = l / NPP;
      const double* ip = w0 + s * NPP * Q2 + l1;
      double v = 0.0;
      for (int q2 = 0; q2 < Q2; ++q2) v += P2[q2 * NPP + l2] * ip[q2 * NPP];
      w1[it] = v;
    }
    __syncthreads();
    // the two layers of direction d are disjoint (NPP >= 2)
    for (int it = tid; it < 2 * NPP * NPP; it += kDgThreads) {
      const int s = it / (NPP * NPP), l = it - s * NPP * NPP;
      acc[layer_node<NPP>(d, s, l % NPP, l / NPP)] += w1[it];
    }
    __syncthreads();
  }
  double* oe = A.out + e * NP3;
  for (int B = tid; B < NP3; B += kDgThreads) oe[B] = acc[B];
}

// ---------------------------------------------------------------------------
// Pressure gradient: out = P p (velocity layout, enrichment rows included).
template <int NPU, int NPP, int NQ, int NQY, bool ENR>
__global__ __launch_bounds__(kDgThreads) void gradient_kernel(const DgArgs A, int layer_lo, int nlayers) {
  constexpr int NU3 = NPU * NPU * NPU, NP3 = NPP * NPP * NPP, NPT = NQ * NQY * NQ;
  __shared__ DgTab<NPU, NPP, NQ, NQY> T;
  __shared__ double sp[NP3];
  __shared__ double w0[3 * NPT], w1[3 * NPT];
  __shared__ double acc[3 * NU3];
  __shared__ double red[3 * (kDgThreads / 64)];
  __shared__ double accE[3];
  const int tid = threadIdx.x;
  int64_t e;
  if (ENR) {
    const int64_t b = blockIdx.x;
    const int ex = (int)(b % A.nx);
    const int64_t t0 = b / A.nx;
    const int slot = (int)(t0 % A.nslots);
    const int ez = (int)(t0 / A.nslots);
    const int ey = slot == A.lower_slot ? 0 : A.ny - 1;
    e = ex + (int64_t)A.nx * (ey + (int64_t)A.ny * ez);
  } else {
    const int64_t b = blockIdx.x;
    const int ex = (int)(b % A.nx);
    const int64_t t0 = b / A.nx;
    e = ex + (int64_t)A.nx * (layer_lo + (int)(t0 % nlayers) + (int64_t)A.ny * (t0 / nlayers));
  }
  const CellGeo g = cell_geo(A, e);
  load_dgtab<NPU, NPP, NQ, NQY, ENR>(A, T, tid);
  const double* pe = A.in + e * NP3;
  for (int i = tid; i < NP3; i += kDgThreads) sp[i] = pe[i];
  __syncthreads();
  const double detJ = g.h[0] * g.h[1] * g.h[2];
  // ---- volume: p at the points, g_c = -(d_c N^u)^T (w |J| p) / h_c
  {
    sweepm<1, 0, NPP, NPP, NPP, NQ, false>(sp, w0, T.Sp, T.Sp, T.Sp, tid);      // [k][j][qx]
    __syncthreads();
    sweepm<1, 1, NQ, NPP, NPP, NQY, false>(w0, w1, T.Spy, T.Spy, T.Spy, tid);  // [k][qy][qx]
    __syncthreads();
    sweepm<1, 2, NQ, NQY, NPP, NQ, false>(w1, w0, T.Sp, T.Sp, T.Sp, tid);      // [qz][qy][qx]
    __syncthreads();
    double ve[3] = {0.0, 0.0, 0.0};
    for (int q = tid; q < NPT; q += kDgThreads) {
      const int qx = q % NQ, qy = (q / NQ) % NQY, qz = q / (NQ * NQY);
      const double v = -T.W[qx] * T.Wy[qy] * T.W[qz] * detJ * w0[q];
      if (ENR) {
        const double* ps = A.psi + (g.enr * A.psi_pts + q) * 4;
        ve[0] += ps[1] * v;
        ve[1] += ps[2] * v;
        ve[2] += ps[3] * v;
      }
      // three copies scaled by 1/h_c for the three components
      w1[q] = v / g.h[0];
      w1[NPT + q] = v / g.h[1];
      w1[2 * NPT + q] = v / g.h[2];
    }
    if (ENR) {
#pragma unroll
      for (int off = 32; off > 0; off >>= 1)
#pragma unroll
        for (int c = 0; c < 3; ++c) ve[c] += __shfl_down(ve[c], off, 64);
      if ((tid & 63) == 0)
#pragma unroll
        for (int c = 0; c < 3; ++c) red[c * (kDgThreads / 64) + (tid >> 6)] = ve[c];
    }
    __syncthreads();
    if (ENR && tid < 3) {
      double s = 0.0;
      for (int wv = 0; wv < kDgThreads / 64; ++wv) s += red[tid * (kDgThreads / 64) + wv];
      accE[tid] = s;
    }
    sweepm<3, 0, NQ, NQY, NQ, NPU, true>(w1, w0, T.Du, T.Su, T.Su, tid);       // [c][qz][qy][i]
    __syncthreads();
    sweepm<3, 1, NPU, NQY, NQ, NPU, true>(w0, w1, T.Suy, T.Duy, T.Suy, tid);   // [c][qz][j][i]
    __syncthreads();
    sweepm<3, 2, NPU, NPU, NQ, NPU, true>(w1, acc, T.Su, T.Su, T.Du, tid);     // [c][k][j][i]
    __syncthreads();
  }
  // ---- faces: (v . n, {{p}}) on the velocity face layer of component d
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
    const int Q1 = t1 == 1 ? NQY : NQ, Q2 = t2 == 1 ? NQY : NQ;
    int nbi[3];
    int64_t nb[2];
    for (int s = 0; s < 2; ++s) nb[s] = neighbour(A, g, d, s, nbi[0], nbi[1], nbi[2]);
    // pressure layers [s][side][l1 + NPP l2]; a wall repeats the own layer (p+ = p-)
    for (int it = tid; it < 4 * NPP * NPP; it += kDgThreads) {
      const int r = it / (NPP * NPP), l = it - r * NPP * NPP;
      const int s = r >> 1, side = r & 1;
      const int l1 = l % NPP, l2 = l / NPP;
      double v;
      if (side == 0 || nb[s] < 0) v = sp[layer_node<NPP>(d, s, l1, l2)];
      else v = A.in[nb[s] * NP3 + layer_node<NPP>(d, 1 - s, l1, l2)];
      w0[it] = v;
    }
    __syncthreads();
    const double* P1 = t1 == 1 ? T.Spy : T.Sp;
    const double* P2 = t2 == 1 ? T.Spy : T.Sp;
    for (int it = tid; it < 4 * Q1 * NPP; it += kDgThreads) {
      const int r = it / (Q1 * NPP), l = it - r * Q1 * NPP;
      const int q1 = l % Q1, l2 = l / Q1;
      const double* ip = w0 + r * NPP * NPP + NPP * l2;
      double s = 0.0;
      for (int l1 = 0; l1 < NPP; ++l1) s += P1[q1 * NPP + l1] * ip[l1];
      w1[it] = s;
    }
    __syncthreads();
    const double area = g.h[t1] * g.h[t2];
    const double* W1 = t1 == 1 ? T.Wy : T.W;
    const double* W2 = t2 == 1 ? T.Wy : T.W;
    double ve[2] = {0.0, 0.0};
    for (int it = tid; it < 2 * Q1 * Q2; it += kDgThreads) {
      const int s = it / (Q1 * Q2), pt = it - s * Q1 * Q2;
      const int q1 = pt % Q1, q2 = pt / Q1;
      double pm = 0.0, pp = 0.0;
      const double* im = w1 + (s * 2 + 0) * Q1 * NPP + q1;
      const double* ipp = w1 + (s * 2 + 1) * Q1 * NPP + q1;
      for (int l2 = 0; l2 < NPP; ++l2) {
        pm += P2[q2 * NPP + l2] * im[l2 * Q1];
        pp += P2[q2 * NPP + l2] * ipp[l2 * Q1];
      }
      const double fl = W1[q1] * W2[q2] * area * (s ? 0.5 : -0.5) * (pm + pp);
      w0[it] = fl;
      if (ENR) ve[s] += A.psi[(g.enr * A.psi_pts + A.psi_off[1 + 2 * d + s] + pt) * 4] * fl;
    }
    if (ENR) {
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) {
        ve[0] += __shfl_down(ve[0], off, 64);
        ve[1] += __shfl_down(ve[1], off, 64);
      }
      if ((tid & 63) == 0) {
        red[tid >> 6] = ve[0];
        red[kDgThreads / 64 + (tid >> 6)] = ve[1];
      }
    }
    __syncthreads();
    if (ENR && tid == 0) {
      double s = 0.0;
      for (int wv = 0; wv < kDgThreads / 64; ++wv) s += red[wv];
      for (int wv = 0; wv < kDgThreads / 64; ++wv) s += red[kDgThreads / 64 + wv];
      accE[d] += s;
    }
    // integrate against the velocity face layer: [s][l1 + NPU l2]
    const double* U1 = t1 == 1 ? T.Suy : T.Su;
    const double* U2 = t2 == 1 ? T.Suy : T.Su;
    for (int it = tid; it < 2 * NPU * Q2; it += kDgThreads) {
      const int s = it / (NPU * Q2), l = it - s * NPU * Q2;
      const int l1 = l % NPU, q2 = l / NPU;
      const double* ip = w0 + s * Q1 * Q2 + Q1 * q2;
      double v = 0.0;
      for (int q1 = 0; q1 < Q1; ++q1) v += U1[q1 * NPU + l1] * ip[q1];
      w1[it] = v;
    }
    __syncthreads();
    for (int it = tid; it < 2 * NPU * NPU; it += kDgThreads) {
      const int s = it / (NPU * NPU), l = it - s * NPU * NPU;
      const int l1 = l % NPU, l2 = l / NPU;
      const double* ip = w1 + s * NPU * Q2 + l1;
      double v = 0.0;
      for (int q2 = 0; q2 < Q2; ++q2) v += U2[q2 * NPU + l2] * ip[q2 * NPU];
      acc[d * NU3 + layer_node<NPU>(d, s, l1, l2)] += v;
    }
    __syncthreads();
  }
  double* oe = A.out + e * 3 * NU3;
  for (int B = tid; B < 3 * NU3; B += kDgThreads) oe[B] = acc[B];
  if (ENR && tid < 3) A.out[A.ncell * 3 * NU3 + g.enr * 3 + tid] = accE[tid];
}

}  // namespace

// (k_u+1, k_p+1, nq_u, nq_wn) combinations: the velocity ones with k_p = k_u - 1
#define DG_DG_COMBOS(X) X(3, 2, 4, 8) X(3, 2, 4, 4) X(4, 3, 4, 8) X(4, 3, 5, 8) X(4, 3, 5, 5) X(5, 4, 7, 8) X(6, 5, 8, 8)

int launch_divgrad(const dg_mesh* m, bool divergence, const double* in, double* out, hipStream_t s) {
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
  A.tab_u = m->tab_u;
  A.tab_pu = m->tab_pu;
  A.psi = m->psi;
  A.in = in;
  A.out = out;
  const int lo = (m->P.fully_periodic || m->lower_slot < 0) ? 0 : 1;
  const int hi = (m->P.fully_periodic || m->upper_slot < 0) ? m->P.ny - 1 : m->P.ny - 2;
  const int nl = hi - lo + 1;
  const int64_t nreg = nl > 0 ? (int64_t)m->P.nx * nl * m->P.nz : 0;
  const int nqw = m->nenr > 0 ? m->P.nq_wn : m->P.nq_u;
#define LAUNCH(KER, pu, pp, q, w, ENRV, grid, lo_, nl_)                                                 \
  hipLaunchKernelGGL((KER<pu, pp, q, w, ENRV>), dim3((unsigned)(grid)), dim3(kDgThreads), 0, s, A, lo_, nl_)
#define X(pu, pp, q, w)                                                                                  \
  if (m->np_u == pu && m->np_p == pp && m->P.nq_u == q && nqw == w) {                                     \
    if (nreg > 0) {                                                                                      \
      if (divergence) LAUNCH(divergence_kernel, pu, pp, q, q, false, nreg, lo, nl);                       \
      else LAUNCH(gradient_kernel, pu, pp, q, q, false, nreg, lo, nl);                                    \
      const int rc = check_hip(hipGetLastError(), "divergence/gradient kernel launch");                  \
      if (rc) return rc;                                                                                 \
    }                                                                                                    \
    if (m->nenr > 0) {                                                                                   \
      if (divergence) LAUNCH(divergence_kernel, pu, pp, q, w, true, m->nenr, 0, 0);                       \
      else LAUNCH(gradient_kernel, pu, pp, q, w, true, m->nenr, 0, 0);                                    \
    }                                                                                                    \
    return check_hip(hipGetLastError(), "divergence/gradient kernel launch");                            \
  }
  DG_DG_COMBOS(X)
#undef X
#undef LAUNCH
  return set_error(DG_ERR_UNSUPPORTED,
                   "pressure gradient / velocity divergence: (k_u+1, k_p+1, nq_u, nq_wn) combination not compiled");
}

}  // namespace dgwm
