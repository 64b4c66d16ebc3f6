// Tile helpers of the direct projection-step solves: a tile holds NC
// columns (cells, or right-hand sides of cells) of 3 NP^3 nodal values,
// T[k * LD + col] with LD = NC + 2, k = component * NP^3 + node and
// node = ix + NP iy + NP^2 iz.
#pragma once

#include <hip/hip_runtime.h>

namespace dgwm {

constexpr int kSpecThreads = 256;

// In place along direction DIR of every (cell, component) block of the tile
// T[k * LD + c] (k = component * NP^3 + node, node = ix + NP iy + NP^2 iz).
template <int NP, int NC, int DIR>
__device__ __forceinline__ void tile_sweep(double* T, const double* Mt, int tid) {
  constexpr int NP2 = NP * NP, NP3 = NP2 * NP, LD = NC + 2;
  constexpr int SD = DIR == 0 ? 1 : (DIR == 1 ? NP : NP2);
  for (int it = tid; it < NC * 3 * NP2; it += kSpecThreads) {
    const int c = it % NC;
    const int rest = it / NC;
    const int comp = rest / NP2, l = rest - comp * NP2;
    const int base = DIR == 0 ? l * NP : (DIR == 1 ? (l % NP) + (l / NP) * NP2 : l);
    const int k0 = comp * NP3 + base;
    double v[NP];
#pragma unroll
    for (int i = 0; i < NP; ++i) v[i] = T[(k0 + i * SD) * LD + c];
#pragma unroll
    for (int a = 0; a < NP; ++a) {
      double o = 0.0;
#pragma unroll
      for (int i = 0; i < NP; ++i) o += Mt[a * NP + i] * v[i];
      T[(k0 + a * SD) * LD + c] = o;
    }
  }
}

// acc[i][j] = sum_k Z[k * N + r_i] T[k * LD + cg * CPT + j], r_i = rl + 64 i.
template <int N, int LD, int RPT, int CPT>
__device__ __forceinline__ void tile_gemm(const double* T, const double* __restrict__ Z, double (&acc)[RPT][CPT],
                                          int rl, int cg) {
#pragma unroll
  for (int i = 0; i < RPT; ++i)
#pragma unroll
    for (int j = 0; j < CPT; ++j) acc[i][j] = 0.0;
#pragma unroll 8
  for (int k = 0; k < N; ++k) {
    double a[CPT];
#pragma unroll
    for (int j = 0; j < CPT; ++j) a[j] = T[k * LD + cg * CPT + j];
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      const int r = rl + 64 * i;
      if (i < RPT - 1 || r < N) {
        const double z = Z[(size_t)k * N + r];
#pragma unroll
        for (int j = 0; j < CPT; ++j) acc[i][j] = fma(z, a[j], acc[i][j]);
      }
    }
  }
}

// Split variant: wavefront wv takes row chunks rw + WR i (rw = wv % WR) and
// the columns cw * CPW .. cw * CPW + CPW - 1 (cw = wv / WR), so each Z entry
// is loaded by 4 / WR wavefronts and each tile value read by WR of them:
// acc[i][j] = sum_k Z[k * N + r_i] T[k * LD + cw * CPW + j], r_i = 64 (rw + WR i) + lane.
template <int N, int LD, int WR, int RPW, int CPW>
__device__ __forceinline__ void tile_gemm_split(const double* T, const double* __restrict__ Z,
                                                double (&acc)[RPW][CPW], int lane, int wv) {
  const int rw = wv % WR, cw = wv / WR;
#pragma unroll
  for (int i = 0; i < RPW; ++i)
#pragma unroll
    for (int j = 0; j < CPW; ++j) acc[i][j] = 0.0;
  int nrow = 0;  // chunks of this wavefront that hold rows
#pragma unroll
  for (int i = 0; i < RPW; ++i)
    if (64 * (rw + WR * i) < N) nrow = i + 1;
#pragma unroll 8
  for (int k = 0; k < N; ++k) {
    double a[CPW];
#pragma unroll
    for (int j = 0; j < CPW; ++j) a[j] = T[k * LD + cw * CPW + j];
#pragma unroll
    for (int i = 0; i < RPW; ++i) {
      const int r = 64 * (rw + WR * i) + lane;
      if (i < nrow) {
        const double z = r < N ? Z[(size_t)k * N + r] : 0.0;
#pragma unroll
        for (int j = 0; j < CPW; ++j) acc[i][j] = fma(z, a[j], acc[i][j]);
      }
    }
  }
}

}  // namespace dgwm
