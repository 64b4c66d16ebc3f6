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

// Vector product: wavefront wv takes row chunks rw + WR i (rw = wv % WR) and
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

typedef double dgwm_d4 __attribute__((ext_vector_type(4)));

// Matrix-core variant for 16-column tiles (FP64 MFMA 16 x 16 x 4): row tile
// t = wv + 4 q of wavefront wv is D = Z^T(rows 16 t .. 16 t + 15) T.  Operand
// lanes: A (Z entries) lane l holds row l % 16, k = k0 + l / 16; B (tile)
// lane l holds k = k0 + l / 16, column l % 16; result element j of lane l is
// row 16 t + 4 j + l / 16, column l % 16.  Rows and k beyond N read zero.
// The operands of the k-steps two ahead are loaded before the current
// step's products are issued.
template <int N, int LD, int RTW>
__device__ __forceinline__ void tile_gemm_mfma(const double* T, const double* __restrict__ Z, dgwm_d4 (&acc)[RTW],
                                               int lane, int wv) {
  constexpr int NT = (N + 15) / 16, NK = (N + 3) / 4;  // row tiles; k-steps
  constexpr int PF = 8;                                 // prefetch depth (k-steps)
#pragma unroll
  for (int q = 0; q < RTW; ++q) acc[q] = dgwm_d4{0.0, 0.0, 0.0, 0.0};
  const int lk = lane >> 4, lr = lane & 15;
  double fa[PF][RTW], fb[PF];
  auto load = [&](int step, double (&a)[RTW], double& b) {
    const int kk = 4 * step + lk;
    const bool kin = step < NK && kk < N;
    b = kin ? T[kk * LD + lr] : 0.0;
#pragma unroll
    for (int q = 0; q < RTW; ++q) {
      const int r = 16 * (wv + 4 * q) + lr;
      a[q] = (kin && r < N) ? Z[(size_t)kk * N + r] : 0.0;
    }
  };
#pragma unroll
  for (int p = 0; p < PF; ++p) load(p, fa[p], fb[p]);
  for (int s0 = 0; s0 < NK; s0 += PF) {
#pragma unroll
    for (int p = 0; p < PF; ++p) {
      double a[RTW], b = fb[p];
#pragma unroll
      for (int q = 0; q < RTW; ++q) a[q] = fa[p][q];
      load(s0 + p + PF, fa[p], fb[p]);
      if (s0 + p < NK) {  // uniform
#pragma unroll
        for (int q = 0; q < RTW; ++q)
          if (wv + 4 * q < NT)  // uniform over the wavefront
            acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[q], b, acc[q], 0, 0, 0);
      }
    }
  }
}

}  // namespace dgwm
