// Geometric multigrid transfers for the pressure operator (preconditioner of
// the Poisson solve; the transfers are the nodal embedding of the coarse DG
// space into the fine one and its transpose).
//
// A coarse cell of level l+1 covers 2 cells of level l along every coarsened
// direction.  Prolongation evaluates the coarse polynomial at the fine cells'
// Gauss-Lobatto nodes, direction by direction:
//   x, z (uniform halves):   child a maps xi_f to xi_c = (a + xi_f) / 2,
//   y (tanh-graded pairs):   with r = h_0 / (h_0 + h_1) of the two fine layers,
//                            child 0: xi_c = r xi_f, child 1: r + (1 - r) xi_f.
// Restriction of residuals (dual vectors) is the transpose.  One workgroup
// per coarse cell; every fine entry has a single writer.
#include <algorithm>
#include <cmath>
#include <vector>

#include "batch.h"

namespace dgwm {

namespace {

// N_i(x) of the NP-node Lobatto basis
template <int NP>
struct LobattoDen {  // 1 / prod_{j != i} (x_i - x_j)
  double inv[NP];
  constexpr LobattoDen() : inv{} {
    for (int i = 0; i < NP; ++i) {
      double d = 1.0;
      for (int j = 0; j < NP; ++j)
        if (j != i) d *= ct::lobatto<NP>.x[i] - ct::lobatto<NP>.x[j];
      inv[i] = 1.0 / d;
    }
  }
};
template <int NP>
inline constexpr LobattoDen<NP> lobatto_den{};

template <int NP>
__device__ __forceinline__ double lobatto_basis(int i, double x) {
  constexpr auto& L = ct::lobatto<NP>;
  double v = lobatto_den<NP>.inv[i];
#pragma unroll
  for (int j = 0; j < NP; ++j)
    if (j != i) v *= x - L.x[j];
  return v;
}

// 1-D prolongation tables P[d][child][l][i] = N_i(xi_c(child, xi_l)) of the
// coarse cell (identity along directions that are not coarsened).
template <typename T, int NP>
__device__ __forceinline__ void build_transfer_tables(T* P, int cx, int cy, int cz, double ry) {
  constexpr auto& L = ct::lobatto<NP>;
  for (int t = threadIdx.x; t < 3 * 2 * NP * NP; t += blockDim.x) {
    const int i = t % NP, l = (t / NP) % NP, ch = (t / (NP * NP)) % 2, d = t / (2 * NP * NP);
    const int c = d == 0 ? cx : (d == 1 ? cy : cz);
    double v;
    if (!c) {
      v = (l == i) ? 1.0 : 0.0;
    } else {
      double xc;
      if (d == 1)
        xc = ch == 0 ? ry * L.x[l] : ry + (1.0 - ry) * L.x[l];
      else
        xc = 0.5 * (ch + L.x[l]);
      v = lobatto_basis<NP>(i, xc);
    }
    P[t] = T(v);
  }
}

// rc = P^T rf on one coarse cell
template <typename T, int NP>
__device__ __forceinline__ void mg_restrict_body(const Tr& tr, int64_t C, const T* __restrict__ rf,
                                                 T* __restrict__ rc) {
  constexpr int NP2 = NP * NP, NP3 = NP2 * NP;
  __shared__ T P[3 * 2 * NP * NP];
  __shared__ T F[8 * NP3];  // [c][b][a][k][j][l]
  __shared__ T G[4 * NP3];  // [c][b][k][j][i]
  __shared__ T H[2 * NP3];  // [c][k][jc][i]
  const int X = (int)(C % tr.ncx), Y = (int)((C / tr.ncx) % tr.ncy), Z = (int)(C / ((int64_t)tr.ncx * tr.ncy));
  const int na = 1 + tr.cx, nb = 1 + tr.cy, nc = 1 + tr.cz;
  const double ry = tr.cy ? tr.hyf[2 * Y] / (tr.hyf[2 * Y] + tr.hyf[2 * Y + 1]) : 0.5;
  build_transfer_tables<T, NP>(P, tr.cx, tr.cy, tr.cz, ry);
  for (int t = threadIdx.x; t < na * nb * nc * NP3; t += blockDim.x) {
    const int node = t % NP3, ch = t / NP3;
    const int a = ch % na, b = (ch / na) % nb, c = ch / (na * nb);
    const int fx = tr.cx ? 2 * X + a : X, fy = tr.cy ? 2 * Y + b : Y, fz = tr.cz ? 2 * Z + c : Z;
    const int64_t fe = fx + (int64_t)tr.nfx * (fy + (int64_t)tr.nfy * fz);
    F[((c * 2 + b) * 2 + a) * NP3 + node] = rf[fe * NP3 + node];
  }
  __syncthreads();
  const T* Px = P;
  const T* Py = P + 2 * NP2;
  const T* Pz = P + 4 * NP2;
  // x: G[c][b][k][j][i] = sum_a sum_l Px[a][l][i] F[c][b][a][k][j][l]
  for (int t = threadIdx.x; t < nc * nb * NP3; t += blockDim.x) {
    const int i = t % NP, kj = (t / NP) % NP2, cb = t / NP3;
    const int b = cb % nb, c = cb / nb;
    T s = 0;
    for (int a = 0; a < na; ++a) {
      const T* f = F + ((c * 2 + b) * 2 + a) * NP3 + kj * NP;
#pragma unroll
      for (int l = 0; l < NP; ++l) s += Px[(a * NP + l) * NP + i] * f[l];
    }
    G[(c * 2 + b) * NP3 + kj * NP + i] = s;
  }
  __syncthreads();
  // y: H[c][k][jc][i] = sum_b sum_m Py[b][m][jc] G[c][b][k][m][i]
  for (int t = threadIdx.x; t < nc * NP3; t += blockDim.x) {
    const int i = t % NP, jc = (t / NP) % NP, k = (t / NP2) % NP, c = t / NP3;
    T s = 0;
    for (int b = 0; b < nb; ++b) {
      const T* g = G + (c * 2 + b) * NP3 + k * NP2 + i;
#pragma unroll
      for (int m = 0; m < NP; ++m) s += Py[(b * NP + m) * NP + jc] * g[m * NP];
    }
    H[c * NP3 + k * NP2 + jc * NP + i] = s;
  }
  __syncthreads();
  // z: rc[kc][jc][i] = sum_c sum_n Pz[c][n][kc] H[c][n][jc][i]
  for (int t = threadIdx.x; t < NP3; t += blockDim.x) {
    const int ji = t % NP2, kc = t / NP2;
    T s = 0;
    for (int c = 0; c < nc; ++c) {
      const T* h = H + c * NP3 + ji;
#pragma unroll
      for (int n = 0; n < NP; ++n) s += Pz[(c * NP + n) * NP + kc] * h[n * NP2];
    }
    rc[C * NP3 + t] = s;
  }
}

// xo = xf + P xc on the fine cells of one coarse cell (xo may be xf: each
// entry is read and written by the same thread)
template <typename T, int NP>
__device__ __forceinline__ void mg_prolong_body(const Tr& tr, int64_t C, const T* __restrict__ xc, const T* xf,
                                                T* xo) {
  constexpr int NP2 = NP * NP, NP3 = NP2 * NP;
  __shared__ T P[3 * 2 * NP * NP];
  __shared__ T S[NP3];      // [kc][jc][i]
  __shared__ T A[2 * NP3];  // [c][n][jc][i]
  __shared__ T B[4 * NP3];  // [c][b][n][m][i]
  const int X = (int)(C % tr.ncx), Y = (int)((C / tr.ncx) % tr.ncy), Z = (int)(C / ((int64_t)tr.ncx * tr.ncy));
  const int na = 1 + tr.cx, nb = 1 + tr.cy, nc = 1 + tr.cz;
  const double ry = tr.cy ? tr.hyf[2 * Y] / (tr.hyf[2 * Y] + tr.hyf[2 * Y + 1]) : 0.5;
  build_transfer_tables<T, NP>(P, tr.cx, tr.cy, tr.cz, ry);
  for (int t = threadIdx.x; t < NP3; t += blockDim.x) S[t] = xc[C * NP3 + t];
  __syncthreads();
  const T* Px = P;
  const T* Py = P + 2 * NP2;
  const T* Pz = P + 4 * NP2;
  for (int t = threadIdx.x; t < nc * NP3; t += blockDim.x) {
    const int ji = t % NP2, n = (t / NP2) % NP, c = t / NP3;
    T s = 0;
#pragma unroll
    for (int k = 0; k < NP; ++k) s += Pz[(c * NP + n) * NP + k] * S[k * NP2 + ji];
    A[c * NP3 + n * NP2 + ji] = s;
  }
  __syncthreads();
  for (int t = threadIdx.x; t < nc * nb * NP3; t += blockDim.x) {
    const int i = t % NP, m = (t / NP) % NP, n = (t / NP2) % NP, cb = t / NP3;
    const int b = cb % nb, c = cb / nb;
    T s = 0;
#pragma unroll
    for (int j = 0; j < NP; ++j) s += Py[(b * NP + m) * NP + j] * A[c * NP3 + n * NP2 + j * NP + i];
    B[(c * 2 + b) * NP3 + n * NP2 + m * NP + i] = s;
  }
  __syncthreads();
  for (int t = threadIdx.x; t < na * nb * nc * NP3; t += blockDim.x) {
    const int node = t % NP3, ch = t / NP3;
    const int a = ch % na, b = (ch / na) % nb, c = ch / (na * nb);
    const int l = node % NP, nm = node / NP;
    T s = 0;
    const T* bb = B + (c * 2 + b) * NP3 + nm * NP;
#pragma unroll
    for (int i = 0; i < NP; ++i) s += Px[(a * NP + l) * NP + i] * bb[i];
    const int fx = tr.cx ? 2 * X + a : X, fy = tr.cy ? 2 * Y + b : Y, fz = tr.cz ? 2 * Z + c : Z;
    const int64_t fe = fx + (int64_t)tr.nfx * (fy + (int64_t)tr.nfy * fz);
    xo[fe * NP3 + node] = xf[fe * NP3 + node] + s;
  }
}

// ---- levels coarsened along all three directions (the usual case) ----
// Several coarse cells per workgroup, one thread per line of every sweep,
// the x and z tables (uniform halves) as compile-time constants, the y table
// of each coarse cell built in LDS, coalesced runs for the fine data.

template <int NP>
constexpr double lagrange_at(int i, double x) {
  double v = 1.0;
  for (int j = 0; j < NP; ++j)
    if (j != i) v *= (x - ct::lobatto<NP>.x[j]) / (ct::lobatto<NP>.x[i] - ct::lobatto<NP>.x[j]);
  return v;
}
// H[a][l][i] = N_i((a + x_l) / 2): child a of a uniformly halved direction
template <int NP>
struct HalfTab {
  double v[2][NP][NP];
  constexpr HalfTab() : v{} {
    for (int a = 0; a < 2; ++a)
      for (int l = 0; l < NP; ++l)
        for (int i = 0; i < NP; ++i) v[a][l][i] = lagrange_at<NP>(i, 0.5 * (a + ct::lobatto<NP>.x[l]));
  }
};
template <int NP>
inline constexpr HalfTab<NP> half_tab{};

constexpr int64_t kFullMinCells = 4096;  // coarse cells from which the batched transfer kernels pay off

template <int NP>
struct Full {
  static constexpr int NP2 = NP * NP, NP3 = NP2 * NP;
  static constexpr int TPC = 4 * NP2;                       // threads per coarse cell (x-sweep lines)
  static constexpr int CPC = 256 / TPC > 0 ? 256 / TPC : 1;  // coarse cells per workgroup
};

// Py[b][m][jc] of coarse cell cc into LDS (2 NP^2 entries per cell)
template <typename T, int NP>
__device__ __forceinline__ void build_py(T* Py, const Tr& tr, int64_t C0, int64_t ncc) {
  constexpr int NP2 = NP * NP, CPC = Full<NP>::CPC;
  constexpr auto& L = ct::lobatto<NP>;
  for (int t = threadIdx.x; t < CPC * 2 * NP2; t += blockDim.x) {
    const int cc = t / (2 * NP2), r = t % (2 * NP2);
    const int jc = r % NP, m = (r / NP) % NP, b = r / NP2;
    const int64_t C = C0 + cc;
    double v = 0.0;
    if (C < ncc) {
      const int Y = ((int)C / tr.ncx) % tr.ncy;
      const double h0 = tr.hyf[2 * Y], ry = h0 / (h0 + tr.hyf[2 * Y + 1]);
      const double xc = b == 0 ? ry * L.x[m] : ry + (1.0 - ry) * L.x[m];
      v = lobatto_basis<NP>(jc, xc);
    }
    Py[cc * 2 * NP2 + (b * NP + m) * NP + jc] = T(v);
  }
}

// first entry of every child (a, b, c) of the workgroup's coarse cells
// (-1 past the last coarse cell); cell counts stay below 2^31
template <int NP>
__device__ __forceinline__ void child_offsets(int64_t* off, const Tr& tr, int64_t C0, int64_t ncc) {
  constexpr int NP3 = NP * NP * NP, CPC = Full<NP>::CPC;
  for (int t = threadIdx.x; t < CPC * 8; t += blockDim.x) {
    const int cc = t / 8, ch = t % 8, a = ch % 2, b = (ch / 2) % 2, c = ch / 4;
    const int64_t C = C0 + cc;
    if (C >= ncc) {
      off[t] = -1;
      continue;
    }
    const int Ci = (int)C, X = Ci % tr.ncx, YZ = Ci / tr.ncx, Y = YZ % tr.ncy, Z = YZ / tr.ncy;
    const int fe = (2 * X + a) + tr.nfx * ((2 * Y + b) + tr.nfy * (2 * Z + c));
    off[t] = (int64_t)fe * NP3;
  }
}

// rc = P^T rf
template <typename T, int NP>
__device__ __forceinline__ void mg_restrict_full_body(const Tr& tr, int64_t ncc, int64_t blk,
                                                      const T* __restrict__ rf, T* __restrict__ rc) {
  using F = Full<NP>;
  constexpr int NP2 = F::NP2, NP3 = F::NP3, CPC = F::CPC;
  __shared__ T sF[CPC * 8 * NP3];  // [cc][c][b][a][k][j][l]
  __shared__ T sG[CPC * 4 * NP3];  // [cc][c][b][k][j][i]
  __shared__ T sH[CPC * 2 * NP3];  // [cc][c][k][jc][i]
  __shared__ T sPy[CPC * 2 * NP2];
  __shared__ int64_t sOff[CPC * 8];
  const int64_t C0 = blk * CPC;
  build_py<T, NP>(sPy, tr, C0, ncc);
  child_offsets<NP>(sOff, tr, C0, ncc);
  __syncthreads();
  // children: (a, node) runs are contiguous in memory
  for (int t = threadIdx.x; t < CPC * 8 * NP3; t += blockDim.x) {
    const int64_t o = sOff[t / NP3];
    sF[t] = o >= 0 ? rf[o + t % NP3] : T(0);
  }
  __syncthreads();
  constexpr auto& H = half_tab<NP>;
  // x: G[c][b][k][j][i] = sum_a sum_l H[a][l][i] F[c][b][a][k][j][l]
  for (int t = threadIdx.x; t < CPC * 4 * NP2; t += blockDim.x) {
    const int cc = t / (4 * NP2), line = t % (4 * NP2);  // line = (c b k j), j fastest
    const int kj = line % NP2, cb = line / NP2;
    const T* f = sF + cc * 8 * NP3 + cb * 2 * NP3 + kj * NP;
    T in[2][NP];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int l = 0; l < NP; ++l) in[a][l] = f[a * NP3 + l];
    T* g = sG + cc * 4 * NP3 + cb * NP3 + kj * NP;
#pragma unroll
    for (int i = 0; i < NP; ++i) {
      T v = 0;
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int l = 0; l < NP; ++l) v += T(H.v[a][l][i]) * in[a][l];
      g[i] = v;
    }
  }
  __syncthreads();
  // y: Hy[c][k][jc][i] = sum_b sum_m Py[b][m][jc] G[c][b][k][m][i]
  for (int t = threadIdx.x; t < CPC * 2 * NP2; t += blockDim.x) {
    const int cc = t / (2 * NP2), line = t % (2 * NP2);  // (c k i), i fastest
    const int i = line % NP, k = (line / NP) % NP, c = line / NP2;
    const T* py = sPy + cc * 2 * NP2;
    T in[2][NP];
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int m = 0; m < NP; ++m) in[b][m] = sG[cc * 4 * NP3 + (c * 2 + b) * NP3 + k * NP2 + m * NP + i];
#pragma unroll
    for (int jc = 0; jc < NP; ++jc) {
      T v = 0;
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int m = 0; m < NP; ++m) v += py[(b * NP + m) * NP + jc] * in[b][m];
      sH[cc * 2 * NP3 + c * NP3 + k * NP2 + jc * NP + i] = v;
    }
  }
  __syncthreads();
  // z: rc[kc][jc][i] = sum_c sum_n H[c][n][kc] Hy[c][n][jc][i]
  for (int t = threadIdx.x; t < CPC * NP2; t += blockDim.x) {
    const int cc = t / NP2, ji = t % NP2;
    const int64_t C = C0 + cc;
    if (C >= ncc) continue;
    T in[2][NP];
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int n = 0; n < NP; ++n) in[c][n] = sH[cc * 2 * NP3 + c * NP3 + n * NP2 + ji];
#pragma unroll
    for (int kc = 0; kc < NP; ++kc) {
      T v = 0;
#pragma unroll
      for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int n = 0; n < NP; ++n) v += T(H.v[c][n][kc]) * in[c][n];
      rc[C * NP3 + kc * NP2 + ji] = v;
    }
  }
}

// xo = xf + P xc (xo may be xf: each entry is read and written by the same thread)
template <typename T, int NP>
__device__ __forceinline__ void mg_prolong_full_body(const Tr& tr, int64_t ncc, int64_t blk,
                                                     const T* __restrict__ xc, const T* xf, T* xo) {
  using F = Full<NP>;
  constexpr int NP2 = F::NP2, NP3 = F::NP3, CPC = F::CPC;
  __shared__ T sS[CPC * NP3];      // [cc][kc][jc][i]
  __shared__ T sA[CPC * 2 * NP3];  // [cc][c][n][jc][i]
  __shared__ T sB[CPC * 4 * NP3];  // [cc][c][b][n][m][i]
  __shared__ T sF[CPC * 8 * NP3];  // [cc][c][b][a][n][m][l]
  __shared__ T sPy[CPC * 2 * NP2];
  __shared__ int64_t sOff[CPC * 8];
  const int64_t C0 = blk * CPC;
  build_py<T, NP>(sPy, tr, C0, ncc);
  child_offsets<NP>(sOff, tr, C0, ncc);
  for (int t = threadIdx.x; t < CPC * NP3; t += blockDim.x) {
    const int64_t C = C0 + t / NP3;
    sS[t] = C < ncc ? xc[C0 * NP3 + t] : T(0);
  }
  __syncthreads();
  constexpr auto& H = half_tab<NP>;
  // z: A[c][n][jc][i] = sum_kc H[c][n][kc] S[kc][jc][i]
  for (int t = threadIdx.x; t < CPC * NP2; t += blockDim.x) {
    const int cc = t / NP2, ji = t % NP2;
    T in[NP];
#pragma unroll
    for (int k = 0; k < NP; ++k) in[k] = sS[cc * NP3 + k * NP2 + ji];
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int n = 0; n < NP; ++n) {
        T v = 0;
#pragma unroll
        for (int k = 0; k < NP; ++k) v += T(H.v[c][n][k]) * in[k];
        sA[cc * 2 * NP3 + c * NP3 + n * NP2 + ji] = v;
      }
  }
  __syncthreads();
  // y: B[c][b][n][m][i] = sum_jc Py[b][m][jc] A[c][n][jc][i]
  for (int t = threadIdx.x; t < CPC * 2 * NP2; t += blockDim.x) {
    const int cc = t / (2 * NP2), line = t % (2 * NP2);  // (c n i), i fastest
    const int i = line % NP, n = (line / NP) % NP, c = line / NP2;
    const T* py = sPy + cc * 2 * NP2;
    T in[NP];
#pragma unroll
    for (int j = 0; j < NP; ++j) in[j] = sA[cc * 2 * NP3 + c * NP3 + n * NP2 + j * NP + i];
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int m = 0; m < NP; ++m) {
        T v = 0;
#pragma unroll
        for (int j = 0; j < NP; ++j) v += py[(b * NP + m) * NP + j] * in[j];
        sB[cc * 4 * NP3 + (c * 2 + b) * NP3 + n * NP2 + m * NP + i] = v;
      }
  }
  __syncthreads();
  // x: F[c][b][a][n][m][l] = sum_i H[a][l][i] B[c][b][n][m][i]
  for (int t = threadIdx.x; t < CPC * 4 * NP2; t += blockDim.x) {
    const int cc = t / (4 * NP2), line = t % (4 * NP2);  // (c b n m), m fastest
    const int nm = line % NP2, cb = line / NP2;
    T in[NP];
#pragma unroll
    for (int i = 0; i < NP; ++i) in[i] = sB[cc * 4 * NP3 + cb * NP3 + nm * NP + i];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int l = 0; l < NP; ++l) {
        T v = 0;
#pragma unroll
        for (int i = 0; i < NP; ++i) v += T(H.v[a][l][i]) * in[i];
        sF[cc * 8 * NP3 + (cb * 2 + a) * NP3 + nm * NP + l] = v;
      }
  }
  __syncthreads();
  for (int t = threadIdx.x; t < CPC * 8 * NP3; t += blockDim.x) {
    const int64_t o0 = sOff[t / NP3];
    if (o0 < 0) continue;
    const int64_t o = o0 + t % NP3;
    xo[o] = xf[o] + sF[t];
  }
}

// x = B b for a dense symmetric B (n x n, n <= kMaxCoarseDofs): one
// wavefront per row, lanes stride along the row (coalesced), two partial sums
// per lane and a butterfly reduction over the wavefront; four rows per
// workgroup, so n / 4 workgroups share the matrix read.
template <typename T>
__device__ __forceinline__ void dense_apply_body(int n, int64_t blk, const T* __restrict__ B, const T* __restrict__ b,
                                                 T* __restrict__ x) {
  const int lane = threadIdx.x & 63;
  const int i = (int)blk * 4 + (threadIdx.x >> 6);
  if (i >= n) return;  // whole wavefronts leave together
  const T* row = B + (int64_t)i * n;
  T s0 = 0, s1 = 0;
  int j = lane;
  for (; j + 64 < n; j += 128) {
    s0 += row[j] * b[j];
    s1 += row[j + 64] * b[j + 64];
  }
  if (j < n) s0 += row[j] * b[j];
  T v = s0 + s1;
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  if (lane == 0) x[i] = v;
}

// Single-mesh kernels (one coarse cell, or CPC coarse cells, per workgroup)
// and their batched forms over many meshes (segment lookup per workgroup).
template <typename T, int NP>
__global__ __launch_bounds__(256) void mg_restrict_kernel(const Tr tr, const T* __restrict__ rf, T* __restrict__ rc) {
  mg_restrict_body<T, NP>(tr, (int64_t)blockIdx.x, rf, rc);
}
template <typename T, int NP>
__global__ __launch_bounds__(256) void mg_prolong_kernel(const Tr tr, const T* __restrict__ xc, const T* xf, T* xo) {
  mg_prolong_body<T, NP>(tr, (int64_t)blockIdx.x, xc, xf, xo);
}
template <typename T, int NP>
__global__ __launch_bounds__(256) void mg_restrict_full(const Tr tr, int64_t ncc, const T* __restrict__ rf,
                                                        T* __restrict__ rc) {
  mg_restrict_full_body<T, NP>(tr, ncc, (int64_t)blockIdx.x, rf, rc);
}
template <typename T, int NP>
__global__ __launch_bounds__(256) void mg_prolong_full(const Tr tr, int64_t ncc, const T* __restrict__ xc,
                                                       const T* xf, T* xo) {
  mg_prolong_full_body<T, NP>(tr, ncc, (int64_t)blockIdx.x, xc, xf, xo);
}
template <typename T>
__global__ __launch_bounds__(256) void dense_apply_kernel(int n, const T* __restrict__ B, const T* __restrict__ b,
                                                          T* __restrict__ x) {
  dense_apply_body<T>(n, (int64_t)blockIdx.x, B, b, x);
}

template <typename T, int NP, bool FULL, bool RESTRICT>
__global__ __launch_bounds__(256) void mg_transfer_batched(const SegArr<TrSeg<T>, kTrSegs> a) {
  const int si = find_seg(a, (int64_t)blockIdx.x);
  const TrSeg<T>& S = a.s[si];
  const int64_t blk = (int64_t)blockIdx.x - S.blk0;
  if (FULL) {
    if (RESTRICT) mg_restrict_full_body<T, NP>(S.tr, S.ncc, blk, S.in, S.out);
    else mg_prolong_full_body<T, NP>(S.tr, S.ncc, blk, S.in, S.add, S.out);
  } else {
    if (RESTRICT) mg_restrict_body<T, NP>(S.tr, blk, S.in, S.out);
    else mg_prolong_body<T, NP>(S.tr, blk, S.in, S.add, S.out);
  }
}

template <typename T>
__global__ __launch_bounds__(256) void dense_apply_batched(const SegArr<DenseSeg<T>, kDenseSegs> a) {
  const int si = find_seg(a, (int64_t)blockIdx.x);
  const DenseSeg<T>& S = a.s[si];
  dense_apply_body<T>((int)S.n, (int64_t)blockIdx.x - S.blk0, S.B, S.b, S.x);
}

// columns of the n x n identity, one vector of n entries per column
__global__ void identity_kernel(double* __restrict__ E, int64_t n) {
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n * n; t += (int64_t)gridDim.x * blockDim.x)
    E[t] = (t / n == t % n) ? 1.0 : 0.0;
}

__global__ void to_f32_kernel(float* __restrict__ o, const double* __restrict__ a, int64_t n) {
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x)
    o[t] = (float)a[t];
}

}  // namespace

Tr mg_transfer_geometry(const dg_mesh* m, int l) {
  const MgLevel& f = m->mg[l];
  const MgLevel& c = m->mg[l + 1];
  Tr t;
  t.nfx = f.nx;
  t.nfy = f.ny;
  t.nfz = f.nz;
  t.ncx = c.nx;
  t.ncy = c.ny;
  t.ncz = c.nz;
  t.cx = c.cx;
  t.cy = c.cy;
  t.cz = c.cz;
  t.hyf = f.hy;
  return t;
}

#define DG_MG_NP(X) X(2) X(3) X(4) X(5) X(6)

bool mg_full_transfer(const dg_mesh* m, int l) {
  const MgLevel& c = m->mg[l + 1];
  return c.cx && c.cy && c.cz && c.ncell >= kFullMinCells;
}

int mg_cells_per_block(int np, bool full) {
  if (!full) return 1;
#define X(a) \
  if (np == a) return Full<a>::CPC;
  DG_MG_NP(X)
#undef X
  return 0;
}

int dense_rows_per_block() { return 4; }

template <typename T>
static int launch_mg_batched(int np, bool full, bool restrict_, const TrSeg<T>* segs, int nseg, hipStream_t s) {
  const int cpc = mg_cells_per_block(np, full);
  if (cpc <= 0) return set_error(DG_ERR_UNSUPPORTED, "multigrid transfer degree not compiled");
  for (int c0 = 0; c0 < nseg; c0 += kTrSegs) {
    SegArr<TrSeg<T>, kTrSegs> a{};
    a.n = std::min(kTrSegs, nseg - c0);
    int64_t blk = 0;
    for (int i = 0; i < a.n; ++i) {
      a.s[i] = segs[c0 + i];
      a.s[i].blk0 = blk;
      blk += (a.s[i].ncc + cpc - 1) / cpc;
    }
    if (blk == 0) continue;
    const dim3 g((unsigned)blk);
    bool done = false;
#define X(q)                                                                                                   \
    if (np == q) {                                                                                             \
      done = true;                                                                                             \
      if (full && restrict_)                                                                                   \
        hipLaunchKernelGGL((mg_transfer_batched<T, q, true, true>), g, dim3(256), 0, s, a);                     \
      else if (full)                                                                                           \
        hipLaunchKernelGGL((mg_transfer_batched<T, q, true, false>), g, dim3(256), 0, s, a);                    \
      else if (restrict_)                                                                                      \
        hipLaunchKernelGGL((mg_transfer_batched<T, q, false, true>), g, dim3(256), 0, s, a);                    \
      else                                                                                                     \
        hipLaunchKernelGGL((mg_transfer_batched<T, q, false, false>), g, dim3(256), 0, s, a);                   \
    }
    DG_MG_NP(X)
#undef X
    if (!done) return set_error(DG_ERR_UNSUPPORTED, "multigrid transfer degree not compiled");
    if (int rc = check_hip(hipGetLastError(), "batched transfer launch")) return rc;
  }
  return DG_OK;
}

template <typename T>
int launch_mg_restrict_batched(int np, bool full, const TrSeg<T>* segs, int nseg, hipStream_t s) {
  return launch_mg_batched<T>(np, full, true, segs, nseg, s);
}
template <typename T>
int launch_mg_prolong_batched(int np, bool full, const TrSeg<T>* segs, int nseg, hipStream_t s) {
  return launch_mg_batched<T>(np, full, false, segs, nseg, s);
}
template <typename T>
int launch_dense_batched(const DenseSeg<T>* segs, int nseg, hipStream_t s) {
  const int rpb = dense_rows_per_block();
  for (int c0 = 0; c0 < nseg; c0 += kDenseSegs) {
    SegArr<DenseSeg<T>, kDenseSegs> a{};
    a.n = std::min(kDenseSegs, nseg - c0);
    int64_t blk = 0;
    for (int i = 0; i < a.n; ++i) {
      a.s[i] = segs[c0 + i];
      a.s[i].blk0 = blk;
      blk += (a.s[i].n + rpb - 1) / rpb;
    }
    if (blk == 0) continue;
    hipLaunchKernelGGL((dense_apply_batched<T>), dim3((unsigned)blk), dim3(256), 0, s, a);
    if (int rc = check_hip(hipGetLastError(), "batched dense apply launch")) return rc;
  }
  return DG_OK;
}
template int launch_mg_restrict_batched<double>(int, bool, const TrSeg<double>*, int, hipStream_t);
template int launch_mg_restrict_batched<float>(int, bool, const TrSeg<float>*, int, hipStream_t);
template int launch_mg_prolong_batched<double>(int, bool, const TrSeg<double>*, int, hipStream_t);
template int launch_mg_prolong_batched<float>(int, bool, const TrSeg<float>*, int, hipStream_t);
template int launch_dense_batched<double>(const DenseSeg<double>*, int, hipStream_t);
template int launch_dense_batched<float>(const DenseSeg<float>*, int, hipStream_t);

int launch_mg_restrict(const dg_mesh* m, int l, dg_prec prec, const void* rf, void* rc, hipStream_t s) {
  const Tr tr = mg_transfer_geometry(m, l);
  const int64_t ncc = m->mg[l + 1].ncell;
  const unsigned nb = (unsigned)ncc;
  // small levels are latency-bound: one workgroup per coarse cell finishes sooner there
  const bool full = mg_full_transfer(m, l);
#define X(a)                                                                                                  \
  if (m->np_p == a && full) {                                                                                 \
    const unsigned g = (unsigned)((ncc + Full<a>::CPC - 1) / Full<a>::CPC);                                   \
    if (prec == DG_F64)                                                                                       \
      hipLaunchKernelGGL((mg_restrict_full<double, a>), dim3(g), dim3(256), 0, s, tr, ncc,                    \
                         static_cast<const double*>(rf), static_cast<double*>(rc));                           \
    else                                                                                                      \
      hipLaunchKernelGGL((mg_restrict_full<float, a>), dim3(g), dim3(256), 0, s, tr, ncc,                     \
                         static_cast<const float*>(rf), static_cast<float*>(rc));                             \
    return check_hip(hipGetLastError(), "restriction launch");                                                \
  }
  DG_MG_NP(X)
#undef X
#define X(a)                                                                                                  \
  if (m->np_p == a) {                                                                                         \
    if (prec == DG_F64)                                                                                       \
      hipLaunchKernelGGL((mg_restrict_kernel<double, a>), dim3(nb), dim3(256), 0, s, tr,                      \
                         static_cast<const double*>(rf), static_cast<double*>(rc));                           \
    else                                                                                                      \
      hipLaunchKernelGGL((mg_restrict_kernel<float, a>), dim3(nb), dim3(256), 0, s, tr,                       \
                         static_cast<const float*>(rf), static_cast<float*>(rc));                             \
    return check_hip(hipGetLastError(), "restriction launch");                                                \
  }
  DG_MG_NP(X)
#undef X
  return set_error(DG_ERR_UNSUPPORTED, "multigrid transfer degree not compiled");
}

int launch_mg_prolong_add(const dg_mesh* m, int l, dg_prec prec, const void* xc, const void* xf, void* xo,
                          hipStream_t s) {
  const Tr tr = mg_transfer_geometry(m, l);
  const int64_t ncc = m->mg[l + 1].ncell;
  const unsigned nb = (unsigned)ncc;
  // small levels are latency-bound: one workgroup per coarse cell finishes sooner there
  const bool full = mg_full_transfer(m, l);
#define X(a)                                                                                                  \
  if (m->np_p == a && full) {                                                                                 \
    const unsigned g = (unsigned)((ncc + Full<a>::CPC - 1) / Full<a>::CPC);                                   \
    if (prec == DG_F64)                                                                                       \
      hipLaunchKernelGGL((mg_prolong_full<double, a>), dim3(g), dim3(256), 0, s, tr, ncc,                     \
                         static_cast<const double*>(xc), static_cast<const double*>(xf),                      \
                         static_cast<double*>(xo));                                                           \
    else                                                                                                      \
      hipLaunchKernelGGL((mg_prolong_full<float, a>), dim3(g), dim3(256), 0, s, tr, ncc,                      \
                         static_cast<const float*>(xc), static_cast<const float*>(xf),                        \
                         static_cast<float*>(xo));                                                            \
    return check_hip(hipGetLastError(), "prolongation launch");                                               \
  }
  DG_MG_NP(X)
#undef X
#define X(a)                                                                                                  \
  if (m->np_p == a) {                                                                                         \
    if (prec == DG_F64)                                                                                       \
      hipLaunchKernelGGL((mg_prolong_kernel<double, a>), dim3(nb), dim3(256), 0, s, tr,                       \
                         static_cast<const double*>(xc), static_cast<const double*>(xf),                      \
                         static_cast<double*>(xo));                                                           \
    else                                                                                                      \
      hipLaunchKernelGGL((mg_prolong_kernel<float, a>), dim3(nb), dim3(256), 0, s, tr,                        \
                         static_cast<const float*>(xc), static_cast<const float*>(xf),                        \
                         static_cast<float*>(xo));                                                            \
    return check_hip(hipGetLastError(), "prolongation launch");                                               \
  }
  DG_MG_NP(X)
#undef X
  return set_error(DG_ERR_UNSUPPORTED, "multigrid transfer degree not compiled");
}

int launch_dense_apply(int64_t n, dg_prec prec, const void* B, const void* b, void* x, hipStream_t s) {
  if (n > kMaxCoarseDofs) return set_error(DG_ERR_ARG, "dense coarse solve larger than its limit");
  const unsigned nb = (unsigned)((n + 3) / 4);  // four rows per workgroup
  if (prec == DG_F64)
    hipLaunchKernelGGL((dense_apply_kernel<double>), dim3(nb), dim3(256), 0, s, (int)n,
                       static_cast<const double*>(B), static_cast<const double*>(b), static_cast<double*>(x));
  else
    hipLaunchKernelGGL((dense_apply_kernel<float>), dim3(nb), dim3(256), 0, s, (int)n, static_cast<const float*>(B),
                       static_cast<const float*>(b), static_cast<float*>(x));
  return check_hip(hipGetLastError(), "dense apply launch");
}

// Levels of a box mesh (host).
int mg_plan(const dg_mesh_params& P, MgLevel* lv) {
  const int np = P.k_p + 1;
  const int64_t np3 = (int64_t)np * np * np;
  int n = 1;
  lv[0] = MgLevel{};
  lv[0].nx = P.nx;
  lv[0].ny = P.ny;
  lv[0].nz = P.nz;
  lv[0].ncell = (int64_t)P.nx * P.ny * P.nz;
  lv[0].n = lv[0].ncell * np3;
  lv[0].hx = P.Lx / P.nx;
  lv[0].hz = P.Lz / P.nz;
  while (n < kMaxLevels) {
    const MgLevel& f = lv[n - 1];
    // small enough for the dense coarse solve: 128 unknowns, or up to
    // 1024 on large meshes (fewer latency-bound tiny levels per V-cycle)
    const int64_t target = std::max<int64_t>(kCoarseTarget, std::min<int64_t>(1024, lv[0].n / 4096));
    if (f.n <= target) break;
    const int cx = (f.nx % 2 == 0) ? 1 : 0;
    const int cy = (f.ny % 2 == 0 && (P.fully_periodic ? f.ny >= 2 : f.ny >= 4)) ? 1 : 0;
    const int cz = (f.nz % 2 == 0) ? 1 : 0;
    if (!cx && !cy && !cz) break;
    MgLevel c{};
    c.cx = cx;
    c.cy = cy;
    c.cz = cz;
    c.nx = cx ? f.nx / 2 : f.nx;
    c.ny = cy ? f.ny / 2 : f.ny;
    c.nz = cz ? f.nz / 2 : f.nz;
    c.ncell = (int64_t)c.nx * c.ny * c.nz;
    c.n = c.ncell * np3;
    c.hx = P.Lx / c.nx;
    c.hz = P.Lz / c.nz;
    lv[n++] = c;
  }
  return n;
}

// Device data of the hierarchy (the pointers of m->mg[] and coarse_inv are
// set by the caller): wall-normal heights of every level from every second
// vertex, Jacobi diagonals, and the pseudo-inverse of the coarsest operator.
// coarse_scr holds 2 n_c^2 doubles of scratch for the assembly.
int mg_setup(dg_mesh* m, const std::vector<double>& eta0, double* coarse_scr, hipStream_t s) {
  int rc = DG_OK;
  std::vector<std::vector<double>> hys(m->mg_nlev);
  std::vector<double> eta = eta0;
  for (int l = 1; l < m->mg_nlev && !rc; ++l) {
    const MgLevel& c = m->mg[l];
    if (c.cy) {
      std::vector<double> e2(c.ny + 1);
      for (int j = 0; j <= c.ny; ++j) e2[j] = eta[2 * j];
      eta.swap(e2);
    }
    hys[l].resize(2 * c.ny);  // heights, then their reciprocals
    for (int j = 0; j < c.ny; ++j) {
      hys[l][j] = eta[j + 1] - eta[j];
      hys[l][c.ny + j] = 1.0 / hys[l][j];
    }
    rc = check_hip(hipMemcpyAsync(m->mg[l].hy, hys[l].data(), sizeof(double) * 2 * c.ny, hipMemcpyHostToDevice, s),
                   "level heights");
    if (!rc) rc = launch_poisson_diag_level(m, l, s);
  }
  if (rc || !m->coarse_inv) {
    if (!rc) rc = check_hip(hipStreamSynchronize(s), "multigrid setup");
    return rc;
  }
  // coarsest operator column by column (A is symmetric), then
  // B = (A + alpha 1 1^T)^{-1}: for b with zero mean, x = B b is the
  // zero-mean solution of A x = b
  const int L = m->mg_nlev - 1;
  const int64_t n = m->mg[L].n;
  double* E = coarse_scr;
  double* Y = coarse_scr + n * n;
  hipLaunchKernelGGL(identity_kernel, dim3(256), dim3(256), 0, s, E, n);
  rc = launch_poisson_level(m, L, DG_F64, E, Y, s, (int)n, n);
  std::vector<double> A(n * n);
  if (!rc) rc = check_hip(hipMemcpyAsync(A.data(), Y, sizeof(double) * n * n, hipMemcpyDeviceToHost, s), "coarse copy");
  if (!rc) rc = check_hip(hipStreamSynchronize(s), "coarse assembly");
  if (rc) return rc;
  double tr = 0;
  for (int64_t i = 0; i < n; ++i) tr += A[i * n + i];
  const double alpha = tr / ((double)n * n);
  for (int64_t i = 0; i < n; ++i)
    for (int64_t j = 0; j < i; ++j) {
      const double v = 0.5 * (A[i * n + j] + A[j * n + i]);
      A[i * n + j] = A[j * n + i] = v;
    }
  for (int64_t t = 0; t < n * n; ++t) A[t] += alpha;
  // Cholesky A = L L^T (lower, in place), W = L^{-1} row by row, then
  // B = W^T W accumulated row by row (all inner loops contiguous)
  for (int64_t j = 0; j < n; ++j) {
    double d = A[j * n + j];
    for (int64_t k = 0; k < j; ++k) d -= A[j * n + k] * A[j * n + k];
    if (!(d > 0)) return set_error(DG_ERR_NONFINITE, "coarsest operator is not positive definite");
    d = std::sqrt(d);
    A[j * n + j] = d;
    const double* Lj = &A[j * n];
    for (int64_t i = j + 1; i < n; ++i) {
      const double* Li = &A[i * n];
      double v = Li[j];
      for (int64_t k = 0; k < j; ++k) v -= Li[k] * Lj[k];
      A[i * n + j] = v / d;
    }
  }
  std::vector<double> W(n * n, 0.0);  // L^{-1}, lower
  for (int64_t i = 0; i < n; ++i) {
    double* Wi = &W[i * n];
    Wi[i] = 1.0;
    for (int64_t k = 0; k < i; ++k) {
      const double lik = A[i * n + k];
      const double* Wk = &W[k * n];
      for (int64_t j = 0; j <= k; ++j) Wi[j] -= lik * Wk[j];
    }
    const double inv = 1.0 / A[i * n + i];
    for (int64_t j = 0; j <= i; ++j) Wi[j] *= inv;
  }
  std::vector<double> B(n * n, 0.0);
  for (int64_t k = 0; k < n; ++k) {
    const double* Wk = &W[k * n];
    for (int64_t i = 0; i <= k; ++i) {
      const double w = Wk[i];
      double* Bi = &B[i * n];
      for (int64_t j = 0; j <= i; ++j) Bi[j] += w * Wk[j];
    }
  }
  for (int64_t i = 0; i < n; ++i)
    for (int64_t j = 0; j < i; ++j) B[j * n + i] = B[i * n + j];
  rc = check_hip(hipMemcpyAsync(m->coarse_inv, B.data(), sizeof(double) * n * n, hipMemcpyHostToDevice, s),
                 "coarse inverse");
  if (!rc) hipLaunchKernelGGL(to_f32_kernel, dim3(256), dim3(256), 0, s, m->coarse_inv32, m->coarse_inv, n * n);
  if (!rc) rc = check_hip(hipStreamSynchronize(s), "multigrid setup");
  return rc;
}

}  // namespace dgwm
