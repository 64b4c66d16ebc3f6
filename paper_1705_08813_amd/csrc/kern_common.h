// Device helpers shared by the operator kernels: mesh arguments and the
// sum-factorization sweep over LDS tiles.
#pragma once

#include <hip/hip_runtime.h>

#include "ctab.h"
#include "dgwm_internal.h"

namespace dgwm {

// Everything a kernel needs about the mesh, passed by value.
struct MeshDev {
  int nx, ny, nz;
  int fully_periodic;
  int lower_slot, upper_slot, nslots;  // enriched-layer slots (-1: wall not enriched)
  double hx, hz;
  const double* hy;   // ny cell heights
  double ihx, ihz;    // 1 / hx, 1 / hz
  const double* ihy;  // ny reciprocal cell heights
  const double* tab;  // 1-D tables (tab_layout)
  const double* psi;  // [enr][psi_pts][4]
  int psi_pts;
  int psi_off[7];     // offsets of volume (0) and faces 0..5 inside one cell's psi table
  double nu, theta;
  double pen;         // ip_factor (k+1)^2
  double wall_mult;
  int64_t enr_off;    // start of the enrichment block in the velocity vector
  // curved geometry (nullptr for affine box cells)
  const double* geo;  // [cell][geo_stride][J^{-1} (9), weight]
  int geo_stride;
  const double* tauF; // [cell][face]
  int nq_wn;          // wall-normal points of enriched cells (the point layout of their tables)
  const double* nut;  // eddy viscosity [enr][psi_pts] of the multiscale viscous operator (else nullptr)
  int ops_off;        // offset of the Poisson operator tables (poi_ops) inside tab
};

// Enriched index of cell (ex, ey, ez) or -1.
__device__ __forceinline__ int64_t enr_index(const MeshDev& M, int ex, int ey, int ez) {
  if (M.fully_periodic) return -1;
  int slot = -1;
  if (ey == 0 && M.lower_slot >= 0) slot = M.lower_slot;
  else if (ey == M.ny - 1 && M.upper_slot >= 0) slot = M.upper_slot;
  if (slot < 0) return -1;
  return ex + M.nx * (slot + M.nslots * ez);  // below 2^31 like the cell count
}

// Apply a 1-D matrix along direction DIR (0 = x fastest) to `ncomp` stacked
// 3-D arrays held in LDS.
//   in : extents (I0, I1, I2), component stride IS
//   out: extent DIR replaced by MO, component stride OS
//   mat: row-major, out = mat * in (mat is MO x NI) or, with TR, out = mat^T in
//        (mat is NI x MO).  ADD accumulates into out.  Every output is scaled.
// One thread per pencil (line along DIR) and component; the pencil is kept in
// registers, the matrix entries are uniform across the wavefront (read from
// LDS as broadcasts when `mat` points there).
template <int DIR, int I0, int I1, int I2, int MO, bool TR, bool ADD, typename T, typename MT>
__device__ __forceinline__ void sweep(const T* __restrict__ in, int IS, T* __restrict__ out, int OS,
                                      const MT* __restrict__ mat, T scale, int ncomp) {
  constexpr int NI = DIR == 0 ? I0 : (DIR == 1 ? I1 : I2);
  constexpr int O0 = DIR == 0 ? MO : I0;
  constexpr int O1 = DIR == 1 ? MO : I1;
  constexpr int P0 = DIR == 0 ? I1 : I0;
  constexpr int P1 = DIR == 2 ? I1 : I2;
  constexpr int NPEN = P0 * P1;
  constexpr int SIN = DIR == 0 ? 1 : (DIR == 1 ? I0 : I0 * I1);
  constexpr int SOUT = DIR == 0 ? 1 : (DIR == 1 ? O0 : O0 * O1);
  for (int t = threadIdx.x; t < NPEN * ncomp; t += blockDim.x) {
    const int c = t / NPEN, p = t - c * NPEN;
    const int a = p % P0, b = p / P0;
    int ib, ob;
    if (DIR == 0) {
      ib = I0 * (a + I1 * b);
      ob = O0 * (a + O1 * b);
    } else if (DIR == 1) {
      ib = a + I0 * I1 * b;
      ob = a + O0 * O1 * b;
    } else {
      ib = a + I0 * b;
      ob = a + O0 * b;
    }
    const T* src = in + c * IS + ib;
    T* dst = out + c * OS + ob;
    T v[NI];
#pragma unroll
    for (int n = 0; n < NI; ++n) v[n] = src[n * SIN];
#pragma unroll
    for (int m = 0; m < MO; ++m) {
      T s = 0;
#pragma unroll
      for (int n = 0; n < NI; ++n) s += T(TR ? mat[n * MO + m] : mat[m * NI + n]) * v[n];
      if (ADD)
        dst[m * SOUT] += scale * s;
      else
        dst[m * SOUT] = scale * s;
    }
  }
}

// As sweep, with a compile-time matrix MAT::at(row, col) (MO x NI, or NI x MO
// with TR): every entry is a literal of the unrolled code.
// The workgroup size NT is a compile-time constant, so a line count below NT
// gives each thread at most one line and the table literals stay local to
// straight-line code.
// tofs rotates the thread-to-line assignment, so that independent sweeps of
// one phase fill the threads a previous sweep left idle.
// With MEM the coefficients are read instead from mp (the same matrix,
// row-major, in device memory): in FP64 a literal costs two scalar moves per
// use, while one wide scalar load brings eight coefficients.
template <int DIR, int I0, int I1, int I2, int MO, bool TR, bool ADD, typename MAT, int NT = 256, bool MEM = false,
          typename T>
__device__ __forceinline__ void sweep_c(const T* __restrict__ in, int IS, T* __restrict__ out, int OS, T scale,
                                        int ncomp, int tofs = 0, const double* __restrict__ mp = nullptr) {
  constexpr int NI = DIR == 0 ? I0 : (DIR == 1 ? I1 : I2);
  constexpr int O0 = DIR == 0 ? MO : I0;
  constexpr int O1 = DIR == 1 ? MO : I1;
  constexpr int P0 = DIR == 0 ? I1 : I0;
  constexpr int P1 = DIR == 2 ? I1 : I2;
  constexpr int NPEN = P0 * P1;
  constexpr int SIN = DIR == 0 ? 1 : (DIR == 1 ? I0 : I0 * I1);
  constexpr int SOUT = DIR == 0 ? 1 : (DIR == 1 ? O0 : O0 * O1);
  const int t0 = (int)threadIdx.x >= tofs ? (int)threadIdx.x - tofs : (int)threadIdx.x + NT - tofs;
  for (int t = t0; t < NPEN * ncomp; t += NT) {
    const int c = t / NPEN, p = t - c * NPEN;
    const int a = p % P0, b = p / P0;
    int ib, ob;
    if (DIR == 0) {
      ib = I0 * (a + I1 * b);
      ob = O0 * (a + O1 * b);
    } else if (DIR == 1) {
      ib = a + I0 * I1 * b;
      ob = a + O0 * O1 * b;
    } else {
      ib = a + I0 * b;
      ob = a + O0 * b;
    }
    const T* src = in + c * IS + ib;
    T* dst = out + c * OS + ob;
    T v[NI];
#pragma unroll
    for (int n = 0; n < NI; ++n) v[n] = src[n * SIN];
#pragma unroll
    for (int m = 0; m < MO; ++m) {
      T s = 0;
#pragma unroll
      for (int n = 0; n < NI; ++n)
        s += T(MEM ? mp[TR ? n * MO + m : m * NI + n] : (TR ? MAT::at(n, m) : MAT::at(m, n))) * v[n];
      if (ADD)
        dst[m * SOUT] += scale * s;
      else
        dst[m * SOUT] = scale * s;
    }
  }
}

// In-place square sweep (MO = NI): every thread reads its whole line into
// registers before writing it back, and lines are disjoint, so input and
// output may be the same array (no __restrict__ here on purpose).
template <int DIR, int I0, int I1, int I2, bool TR, typename MAT, int NT = 256, bool MEM = false, typename T>
__device__ __forceinline__ void sweep_c_inplace(T* a, int IS, T scale, int ncomp, int tofs = 0,
                                                const double* __restrict__ mp = nullptr) {
  constexpr int NI = DIR == 0 ? I0 : (DIR == 1 ? I1 : I2);
  constexpr int P0 = DIR == 0 ? I1 : I0;
  constexpr int P1 = DIR == 2 ? I1 : I2;
  constexpr int NPEN = P0 * P1;
  constexpr int SIN = DIR == 0 ? 1 : (DIR == 1 ? I0 : I0 * I1);
  const int t0 = (int)threadIdx.x >= tofs ? (int)threadIdx.x - tofs : (int)threadIdx.x + NT - tofs;
  for (int t = t0; t < NPEN * ncomp; t += NT) {
    const int c = t / NPEN, p = t - c * NPEN;
    const int aa = p % P0, b = p / P0;
    const int ib = DIR == 0 ? I0 * (aa + I1 * b) : (DIR == 1 ? aa + I0 * I1 * b : aa + I0 * b);
    T* line = a + c * IS + ib;
    T v[NI];
#pragma unroll
    for (int n = 0; n < NI; ++n) v[n] = line[n * SIN];
    T w[NI];
#pragma unroll
    for (int m = 0; m < NI; ++m) {
      T s = 0;
#pragma unroll
      for (int n = 0; n < NI; ++n)
        s += T(MEM ? mp[TR ? n * NI + m : m * NI + n] : (TR ? MAT::at(n, m) : MAT::at(m, n))) * v[n];
      w[m] = scale * s;
    }
#pragma unroll
    for (int m = 0; m < NI; ++m) line[m * SIN] = w[m];
  }
}

// Deterministic block sum of three per-thread partials (fixed order:
// butterfly within each wavefront, then waves in index order).
template <typename T>
__device__ __forceinline__ void block_sum3(T v[3], T* red /* >= 3 * nwaves */) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    T x = v[c];
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o, 64);
    if (lane == 0) red[3 * wave + c] = x;
  }
  __syncthreads();
  if (threadIdx.x < 3) {
    T s = 0;
    for (int w = 0; w < nw; ++w) s += red[3 * w + threadIdx.x];
    v[0] = s;  // thread c holds component c
  }
}

// Workgroup sum of N per-thread values; thread i < N receives sum i in v[0].
template <int N, typename T>
__device__ __forceinline__ void block_sum_n(T* v, T* red /* >= N * nwaves */) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
#pragma unroll
  for (int c = 0; c < N; ++c) {
    T x = v[c];
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o, 64);
    if (lane == 0) red[N * wave + c] = x;
  }
  __syncthreads();
  if (threadIdx.x < N) {
    T s = 0;
    for (int w = 0; w < nw; ++w) s += red[N * w + threadIdx.x];
    v[0] = s;
  }
}

}  // namespace dgwm
