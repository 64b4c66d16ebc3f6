// Direct solve of the element-wise projection step (arXiv 1705.08813, Sec.
// 4.2, eq. projectionspat) in cells without enrichment, FP64.
//
// In a cell of height h_y (flat mesh, affine cell) the system is
//   (M_e + D_e) x = M_e u_hat - s g,   M_e = |J| Mh,   D_e = |J| tau_D,e Dh,
// with Mh the reference mass (the tensor product K (x) K (x) K of the 1-D
// mass K of the velocity rule, per component) and Dh the div-div form with
// physical derivatives and reference weights; Mh and Dh depend on the layer
// only, tau_D,e on the cell.  With the Cholesky factor K = C C^T and
// L = C (x) C (x) C (Mh = L L^T), and the eigendecomposition of the
// whitened form  L^{-1} Dh L^{-T} = Z diag(lambda) Z^T  (once per distinct
// layer height, on the host, by the cyclic Jacobi method),
//   x = L^{-T} Z diag(1 / (1 + tau_D,e lambda)) Z^T L^T (u_hat - (s/|J|) Mh^{-1} g).
// Mh^{-1} is a sweep with 1-D matrices; L^T and L^{-T} are folded into the
// layer's tables, (L Z)^T and L^{-T} Z, which are dense products shared by
// all cells of a layer, so a workgroup takes a tile of NC
// cells of one layer and runs both products out of LDS, on the FP64 matrix
// cores for 16-cell tiles (a vector product for the 8-cell tiles of k = 5).
// The result is exact up to rounding: no iteration, every cell the same work.
#include <algorithm>
#include <thread>
#include <vector>

#include "kern_common.h"
#include "kern_tile.h"
#include "symeig.h"

namespace dgwm {

namespace {


template <int NP>
constexpr int spec_nc() {
  return NP >= 6 ? 8 : 16;
}

struct SpecArgs {
  int nx, ny, layer_lo, tiles, nblocks;  // tiles per layer; blocks in the launch
  int64_t ncol;                          // cells per layer (nx * nz)
  double hx, hz;
  const double* hy;     // [ny] cell heights
  const double* mats;   // [3][np][np]: K^{-1}, C^T, C^{-T} (row-major, out_a = sum_i M[a][i] in_i)
  const double* slots;  // [slot][2 n^2 + n]: A1[k][r] = (L Z)[k][r], A2[k][r] = (L^{-T} Z)[r][k], lambda
  const int32_t* map;   // [ny] slot of each layer
  const double* tau_d;
  const double* u_hat;
  const double* g;
  double scale;
  double* x;
};

template <int NP, int NC>
__global__ __launch_bounds__(kSpecThreads) void spectral_step_kernel(const SpecArgs A) {
  constexpr int NP2 = NP * NP, NP3 = NP2 * NP, N = 3 * NP3, LD = NC + 2;
  constexpr int WR = 2, CPW = NC / (4 / WR);       // wavefronts along rows; columns per wavefront
  constexpr int RPW = ((N + 63) / 64 + WR - 1) / WR;  // row chunks per wavefront
  __shared__ double T[N * LD];
  __shared__ double Mt[3 * NP2];
  __shared__ double tauc[NC];
  // consecutive logical blocks (tiles of one layer) on one XCD: hardware
  // block b runs on XCD b % 8
  const int per = (A.nblocks + 7) / 8;
  const int lb = (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
  if (lb >= A.nblocks) return;
  const int tid = threadIdx.x;
  const int layer = A.layer_lo + lb / A.tiles;
  const int64_t j0 = (int64_t)(lb % A.tiles) * NC;
  const int nc = A.ncol - j0 < NC ? (int)(A.ncol - j0) : NC;
  const int64_t rowc = (int64_t)A.nx * A.ny;
  auto cell = [&](int c) -> int64_t {
    const int64_t j = j0 + c;
    return j % A.nx + (int64_t)A.nx * layer + rowc * (j / A.nx);
  };
  for (int i = tid; i < 3 * NP2; i += kSpecThreads) Mt[i] = A.mats[i];
  if (tid < NC) tauc[tid] = tid < nc ? A.tau_d[cell(tid)] : 0.0;
  const double detJ = A.hx * A.hy[layer] * A.hz;
  for (int idx = tid; idx < NC * N; idx += kSpecThreads) {
    const int c = idx / N, k = idx - c * N;
    T[k * LD + c] = c < nc ? A.g[cell(c) * N + k] : 0.0;
  }
  __syncthreads();
  // Mh^{-1} g
  tile_sweep<NP, NC, 0>(T, Mt, tid);
  __syncthreads();
  tile_sweep<NP, NC, 1>(T, Mt, tid);
  __syncthreads();
  tile_sweep<NP, NC, 2>(T, Mt, tid);
  __syncthreads();
  const double f = A.scale / detJ;
  for (int idx = tid; idx < NC * N; idx += kSpecThreads) {
    const int c = idx / N, k = idx - c * N;
    T[k * LD + c] = (c < nc ? A.u_hat[cell(c) * N + k] : 0.0) - f * T[k * LD + c];
  }
  __syncthreads();
  // (the factors L^T before and L^{-T} after the products are folded into the tables)
  const double* Zs = A.slots + (size_t)A.map[layer] * (2 * (size_t)N * N + N);
  const double* lam = Zs + 2 * (size_t)N * N;
  const int lane = tid & 63, wv = tid >> 6;
  if constexpr (NC == 16) {
    // matrix cores: wavefront wv owns row tiles wv + 4 q, all 16 columns
    constexpr int RTW = ((N + 15) / 16 + 3) / 4;
    dgwm_d4 acc[RTW];
    tile_gemm_mfma<N, LD, RTW>(T, Zs, acc, lane, wv);
    __syncthreads();
#pragma unroll
    for (int q = 0; q < RTW; ++q)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int r = 16 * (wv + 4 * q) + 4 * j + (lane >> 4), c = lane & 15;
        if (r < N) T[r * LD + c] = acc[q][j] / (1.0 + tauc[c] * lam[r]);
      }
    __syncthreads();
    tile_gemm_mfma<N, LD, RTW>(T, Zs + (size_t)N * N, acc, lane, wv);
    __syncthreads();
#pragma unroll
    for (int q = 0; q < RTW; ++q)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int r = 16 * (wv + 4 * q) + 4 * j + (lane >> 4), c = lane & 15;
        if (r < N) T[r * LD + c] = acc[q][j];
      }
  } else {
    const int rw = wv % WR, c0 = (wv / WR) * CPW;
    double acc[RPW][CPW];
    tile_gemm_split<N, LD, WR, RPW, CPW>(T, Zs, acc, lane, wv);
    __syncthreads();
#pragma unroll
    for (int i = 0; i < RPW; ++i) {
      const int r = 64 * (rw + WR * i) + lane;
      if (r < N) {
        const double lr = lam[r];
#pragma unroll
        for (int j = 0; j < CPW; ++j) T[r * LD + c0 + j] = acc[i][j] / (1.0 + tauc[c0 + j] * lr);
      }
    }
    __syncthreads();
    tile_gemm_split<N, LD, WR, RPW, CPW>(T, Zs + (size_t)N * N, acc, lane, wv);
    __syncthreads();
#pragma unroll
    for (int i = 0; i < RPW; ++i) {
      const int r = 64 * (rw + WR * i) + lane;
      if (r < N) {
#pragma unroll
        for (int j = 0; j < CPW; ++j) T[r * LD + c0 + j] = acc[i][j];
      }
    }
    __syncthreads();
  }
  __syncthreads();
  for (int idx = tid; idx < NC * N; idx += kSpecThreads) {
    const int c = idx / N, k = idx - c * N;
    if (c < nc) A.x[cell(c) * N + k] = T[k * LD + c];
  }
}

// Lower Cholesky factor of the symmetric positive definite n x n matrix a.
void cholesky(int n, const std::vector<double>& a, std::vector<double>& c) {
  c.assign((size_t)n * n, 0.0);
  for (int j = 0; j < n; ++j) {
    double d = a[j * n + j];
    for (int k = 0; k < j; ++k) d -= c[j * n + k] * c[j * n + k];
    c[j * n + j] = std::sqrt(d);
    for (int i = j + 1; i < n; ++i) {
      double s = a[i * n + j];
      for (int k = 0; k < j; ++k) s -= c[i * n + k] * c[j * n + k];
      c[i * n + j] = s / c[j * n + j];
    }
  }
}

// Inverse of a lower triangular matrix (forward substitution per column).
void lower_inverse(int n, const std::vector<double>& c, std::vector<double>& ci) {
  ci.assign((size_t)n * n, 0.0);
  for (int col = 0; col < n; ++col) {
    for (int i = col; i < n; ++i) {
      double s = i == col ? 1.0 : 0.0;
      for (int k = col; k < i; ++k) s -= c[i * n + k] * ci[k * n + col];
      ci[i * n + col] = s / c[i * n + i];
    }
  }
}

}  // namespace

int spectral_layers(const dg_mesh& m, std::vector<int>* map, std::vector<double>* heights) {
  const dg_mesh_params& P = m.P;
  if (m.curved) return 0;
  const int lo = 0, hi = P.ny - 1;  // every layer (enriched cells share their polynomial block)
  std::vector<double> hs;
  if (map) map->assign(P.ny, 0);
  for (int j = lo; j <= hi; ++j) {
    const double t0 = 2.0 * j / P.ny - 1.0, t1 = 2.0 * (j + 1) / P.ny - 1.0;
    const double h = P.gamma > 0 ? std::tanh(P.gamma * t1) / std::tanh(P.gamma) - std::tanh(P.gamma * t0) / std::tanh(P.gamma)
                                 : t1 - t0;
    int s = -1;
    for (size_t q = 0; q < hs.size(); ++q)
      if (hs[q] == h) s = (int)q;
    if (s < 0) {
      s = (int)hs.size();
      hs.push_back(h);
    }
    if (map) (*map)[j] = s;
  }
  if (heights) *heights = hs;
  return (int)hs.size();
}

size_t spectral_table_doubles(const dg_mesh& m) {
  const int ns = spectral_layers(m, nullptr, nullptr);
  if (ns == 0) return 0;
  const size_t n = 3 * (size_t)m.np_u * m.np_u * m.np_u;
  return 3 * (size_t)m.np_u * m.np_u + (size_t)ns * (2 * n * n + n) + (m.P.ny + 1) / 2;  // + int32 map
}

// Host: 1-D factors, whitened div-div forms, their eigendecompositions; copies
// everything into m->spec (synchronous on s).
static int build_spectral_tables(const dg_mesh* m, hipStream_t s) {
  const dg_mesh_params& P = m->P;
  const int np = m->np_u, nq = P.nq_u, np3 = np * np * np, n = 3 * np3, npt = nq * nq * nq;
  std::vector<int> map;
  std::vector<double> heights;
  const int ns = spectral_layers(*m, &map, &heights);
  if (ns == 0) return DG_OK;
  const TabLayout Lu = tab_layout(np, nq, P.nq_wn);
  std::vector<double> tu(Lu.size);
  fill_tables(np, nq, P.nq_wn, tu.data());
  const double* S = tu.data() + Lu.S;
  const double* Sd = tu.data() + Lu.Sd;
  const double* w = tu.data() + Lu.w;
  std::vector<double> K((size_t)np * np), C, Ci;
  for (int i = 0; i < np; ++i)
    for (int j = 0; j < np; ++j) {
      double v = 0.0;
      for (int q = 0; q < nq; ++q) v += w[q] * S[q * np + i] * S[q * np + j];
      K[i * np + j] = v;
    }
  cholesky(np, K, C);
  lower_inverse(np, C, Ci);
  const size_t head = 3 * (size_t)np * np, per = 2 * (size_t)n * n + n;
  std::vector<double> host(spectral_table_doubles(*m), 0.0);
  double* Kinv = host.data();
  double* CT = Kinv + np * np;
  double* CiT = CT + np * np;
  for (int a = 0; a < np; ++a)
    for (int i = 0; i < np; ++i) {
      double v = 0.0;  // K^{-1} = C^{-T} C^{-1}
      for (int k = 0; k < np; ++k) v += Ci[k * np + a] * Ci[k * np + i];
      Kinv[a * np + i] = v;
      CT[a * np + i] = C[i * np + a];
      CiT[a * np + i] = Ci[i * np + a];
    }
  // whitened 1-D tables: St = S C^{-T}, Sdt = Sd C^{-T}
  std::vector<double> St((size_t)nq * np, 0.0), Sdt((size_t)nq * np, 0.0);
  for (int q = 0; q < nq; ++q)
    for (int a = 0; a < np; ++a)
      for (int i = 0; i < np; ++i) {
        St[q * np + a] += S[q * np + i] * Ci[a * np + i];
        Sdt[q * np + a] += Sd[q * np + i] * Ci[a * np + i];
      }
  std::vector<int> sweeps(ns, 0);
  auto work = [&](int slot) {
    const double h[3] = {m->hx, heights[slot], m->hz};
    // G[q][I] = sqrt(w_q) div of whitened basis function I at point q
    std::vector<double> G((size_t)npt * n);
    for (int qz = 0; qz < nq; ++qz)
      for (int qy = 0; qy < nq; ++qy)
        for (int qx = 0; qx < nq; ++qx) {
          const int q = qx + nq * (qy + nq * qz);
          const double sw = std::sqrt(w[qx] * w[qy] * w[qz]);
          for (int iz = 0; iz < np; ++iz)
            for (int iy = 0; iy < np; ++iy)
              for (int ix = 0; ix < np; ++ix) {
                const int B = ix + np * (iy + np * iz);
                const double sx = St[qx * np + ix], sy = St[qy * np + iy], sz = St[qz * np + iz];
                G[(size_t)q * n + B] = sw * Sdt[qx * np + ix] * sy * sz / h[0];
                G[(size_t)q * n + np3 + B] = sw * sx * Sdt[qy * np + iy] * sz / h[1];
                G[(size_t)q * n + 2 * np3 + B] = sw * sx * sy * Sdt[qz * np + iz] / h[2];
              }
        }
    std::vector<double> Bm((size_t)n * n, 0.0), lam, vt;
    for (int q = 0; q < npt; ++q) {
      const double* gq = &G[(size_t)q * n];
      for (int I = 0; I < n; ++I) {
        const double gi = gq[I];
        if (gi == 0.0) continue;
        double* row = &Bm[(size_t)I * n];
        for (int J = 0; J < n; ++J) row[J] += gi * gq[J];
      }
    }
    sweeps[slot] = sym_eig_jacobi(n, Bm, lam, vt);
    // first product: (L Z)^T, stored as A1[k][r] = (L z_r)[k]; second: L^{-T} Z, stored as A2[k][r] = (L^{-T} z_k)[r]
    // (z_r eigenvector r; L and L^{-T} applied as 1-D factors along each direction of each component)
    double* A1 = host.data() + head + slot * per;
    double* A2 = A1 + (size_t)n * n;
    double* L = A2 + (size_t)n * n;
    std::vector<double> v((size_t)n), w((size_t)n);
    auto along = [&](const std::vector<double>& M, bool transpose, std::vector<double>& x) {
      for (int dir = 0; dir < 3; ++dir) {
        const int sd = dir == 0 ? 1 : (dir == 1 ? np : np * np);
        for (int c = 0; c < 3; ++c)
          for (int l = 0; l < np * np; ++l) {
            const int base = c * np3 + (dir == 0 ? l * np : (dir == 1 ? (l % np) + (l / np) * np * np : l));
            double in[8], out[8];
            for (int i = 0; i < np; ++i) in[i] = x[base + i * sd];
            for (int a = 0; a < np; ++a) {
              double t = 0.0;
              for (int i = 0; i < np; ++i) t += (transpose ? M[i * np + a] : M[a * np + i]) * in[i];
              out[a] = t;
            }
            for (int a = 0; a < np; ++a) x[base + a * sd] = out[a];
          }
      }
    };
    for (int r = 0; r < n; ++r) {
      for (int k = 0; k < n; ++k) v[k] = w[k] = vt[(size_t)r * n + k];
      along(C, false, v);   // L z_r
      along(Ci, true, w);   // L^{-T} z_r
      for (int k = 0; k < n; ++k) {
        A1[(size_t)k * n + r] = v[k];
        A2[(size_t)r * n + k] = w[k];
      }
    }
    for (int r = 0; r < n; ++r) L[r] = std::max(lam[r], 0.0);  // positive semidefinite form
  };
  // slots t, t + nth, ... per worker; an allocation failure marks the slot (-2) instead of escaping the thread,
  // and workers that cannot be started run on this thread
  auto run = [&](int t, int nth) {
    for (int slot = t; slot < ns; slot += nth) {
      try {
        work(slot);
      } catch (...) {
        sweeps[slot] = -2;
      }
    }
  };
  const int nth = std::max(1, std::min<int>(ns, std::min(16u, std::max(1u, std::thread::hardware_concurrency()))));
  std::vector<std::thread> pool;
  int started = 0;
  try {
    pool.reserve(nth);
    for (; started < nth; ++started) pool.emplace_back(run, started, nth);
  } catch (...) {
  }
  for (int t = started; t < nth; ++t) run(t, nth);
  for (auto& th : pool) th.join();
  for (int slot = 0; slot < ns; ++slot) {
    if (sweeps[slot] == -2) return set_error(DG_ERR_ARG, "projection step: host memory for the layer tables refused");
    if (sweeps[slot] < 0) return set_error(DG_ERR_NOT_CONVERGED, "projection step: eigendecomposition did not converge");
  }
  int32_t* mp = reinterpret_cast<int32_t*>(host.data() + head + ns * per);
  for (int j = 0; j < P.ny; ++j) mp[j] = map[j];
  int rc = check_hip(hipMemcpyAsync(m->spec, host.data(), sizeof(double) * host.size(), hipMemcpyHostToDevice, s),
                     "copy");
  if (!rc) rc = check_hip(hipStreamSynchronize(s), "projection step tables");
  if (!rc) m->spec_ok = 1;
  return rc;
}

int ensure_spectral_tables(const dg_mesh* m, hipStream_t s) {
  if (m->spec_ok) return DG_OK;
  try {
    return build_spectral_tables(m, s);
  } catch (...) {  // host allocations: no exception crosses the C ABI
    return set_error(DG_ERR_ARG, "projection step: host memory for the layer tables refused");
  }
}

void spectral_pointers(const dg_mesh* m, const double** mats, const double** slots, const int32_t** map) {
  const int np = m->np_u;
  const size_t n = 3 * (size_t)np * np * np;
  const int ns = spectral_layers(*m, nullptr, nullptr);
  *mats = m->spec;
  *slots = m->spec + 3 * np * np;
  *map = reinterpret_cast<const int32_t*>(m->spec + 3 * np * np + (size_t)ns * (2 * n * n + n));
}

int launch_spectral_step(const dg_mesh* m, const double* tau_d, const double* u_hat, const double* g, double scale,
                         double* x, hipStream_t s) {
  const dg_mesh_params& P = m->P;
  const int lo = (P.fully_periodic || m->lower_slot < 0) ? 0 : 1;
  const int hi = (P.fully_periodic || m->upper_slot < 0) ? P.ny - 1 : P.ny - 2;
  const int nl = hi - lo + 1;
  if (nl <= 0) return DG_OK;
  const int np = m->np_u;
  SpecArgs A;
  A.nx = P.nx;
  A.ny = P.ny;
  A.layer_lo = lo;
  A.ncol = (int64_t)P.nx * P.nz;
  A.hx = m->hx;
  A.hz = m->hz;
  A.hy = m->hy;
  spectral_pointers(m, &A.mats, &A.slots, &A.map);
  A.tau_d = tau_d;
  A.u_hat = u_hat;
  A.g = g;
  A.scale = scale;
  A.x = x;
#define X(p)                                                                                                \
  if (np == p) {                                                                                            \
    constexpr int nc = spec_nc<p>();                                                                        \
    const int64_t tiles = (A.ncol + nc - 1) / nc;                                                           \
    const int64_t nb = tiles * nl;                                                                          \
    if (nb > INT32_MAX / 2) return set_error(DG_ERR_ARG, "projection step: mesh too large");                \
    A.tiles = (int)tiles;                                                                                   \
    A.nblocks = (int)nb;                                                                                    \
    const int grid = ((A.nblocks + 7) / 8) * 8;                                                             \
    hipLaunchKernelGGL((spectral_step_kernel<p, nc>), dim3((unsigned)grid), dim3(kSpecThreads), 0, s, A);   \
    return check_hip(hipGetLastError(), "projection step kernel launch");                                   \
  }
  X(3) X(4) X(5) X(6)
#undef X
  return set_error(DG_ERR_UNSUPPORTED, "projection step: degree not compiled");
}

}  // namespace dgwm
