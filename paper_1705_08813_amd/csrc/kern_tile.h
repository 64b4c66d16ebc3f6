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
#pragma unroll 2
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

}  // namespace dgwm
