// Helmholtz step of the dual-splitting scheme (arXiv 1705.08813, Sec. 4.1
// eq. visc, Sec. 4.2 eq. helmholtzspat):
//   (gamma0/dt) M u + A(nu_t) u = (gamma0/dt) M u_hathat,
// with A u = -F^nu_e(v, u) the multiscale viscous operator (eq.
// viscous_multiscale, adjoint sign -1: not symmetric) and M the velocity mass
// matrix.  Solved as  H x = gamma x + M^{-1} A x = gamma b  (gamma = gamma0/dt,
// b = u_hathat) by restarted GMRES in FP64: the block-diagonal M^{-1} acts as
// the (left) preconditioner, which leaves an operator close to gamma I for the
// small time steps of the explicit convective step; the paper solves this
// step with GMRES (Sec. 5.1 reports its iteration counts).
//
// The Arnoldi process runs on K = M^{-1} A instead of H = gamma I + K: both
// span the same Krylov spaces, and the Hessenberg matrix of H is that of K
// with gamma added to its diagonal.  This keeps the dominant gamma v_j out of
// the new vector, so its projections do not cancel.  Orthogonalisation is
// classical Gram-Schmidt over all previous basis vectors at once (one pass
// computes every projection, one pass subtracts them and forms the norm),
// repeated once when the norm drops below 1/sqrt(2) of its value before the
// projection (the test of Daniel, Gragg, Kaufman and Stewart, 1976).  Every
// scalar of an Arnoldi step stays on the device (the projections are
// subtracted with their device values) and one copy per step (two with the
// repeat) brings the new Hessenberg column to the host, where the Givens
// rotations and the least-squares solution live.  Reductions are two-stage
// fixed-grid sums (deterministic).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <vector>

#include "dgwm_internal.h"

namespace dgwm {

namespace {

constexpr int kHThreads = 256;
constexpr int kHMaxParts = 1024;
constexpr int kHMaxRestart = 100;
constexpr int kHChunk = 16;      // basis vectors per pass of the multi-vector kernels
// device scalars: the first and the repeated projections of a Hessenberg
// column with their norms (kHPass2 apart), ||w||^2 before the projection,
// ||gamma b||^2 and ||gamma b||
constexpr int kHPass2 = 104;
constexpr int kHScalars = 256;
constexpr int kHSlotW = kHScalars - 3;
constexpr int kHRows = kHMaxRestart + 2;  // rows of reduction partials

int h_blocks(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>((n + 511) / 512, kHMaxParts)); }
unsigned ew_blocks(int64_t n) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 2048)); }

__device__ __forceinline__ double h_block_sum(double v, double* sh) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double s = 0;
  if (threadIdx.x == 0)
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s += sh[i];
  return s;
}

// part[b] = partial sums of a.b
__global__ __launch_bounds__(kHThreads) void h_dot(const double* __restrict__ a, const double* __restrict__ b,
                                                   int64_t n, double* __restrict__ part) {
  __shared__ double sh[kHThreads / 64];
  double v = 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    v += a[i] * b[i];
  v = h_block_sum(v, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = v;
}

// *out = sum of nb partials (fixed order); with sqrt_out, *out2 = sqrt(*out)
__global__ __launch_bounds__(kHThreads) void h_final(const double* __restrict__ part, int nb, double* __restrict__ out,
                                                     double* __restrict__ out2) {
  __shared__ double sh[kHThreads / 64];
  double v = 0;
  for (int i = threadIdx.x; i < nb; i += blockDim.x) v += part[i];
  v = h_block_sum(v, sh);
  if (threadIdx.x == 0) {
    *out = v;
    if (out2) *out2 = sqrt(v);
  }
}

// Projections of w on nk <= kHChunk basis vectors V_k0 .. V_{k0+nk-1} in one
// pass: part[(k0 + k) nbp + b] = block b's partial sum of V_{k0+k} . w, and
// with ww also part[(kHRows - 1) nbp + b] = its partial sum of w . w.
__global__ __launch_bounds__(kHThreads) void h_mdot(const double* __restrict__ V, int64_t stride, int k0, int nk,
                                                    const double* __restrict__ w, int64_t n, double* __restrict__ part,
                                                    int nbp, int ww) {
  __shared__ double sh[(kHChunk + 1) * (kHThreads / 64)];
  double acc[kHChunk + 1];
#pragma unroll
  for (int k = 0; k <= kHChunk; ++k) acc[k] = 0.0;
  const double* v0 = V + (int64_t)k0 * stride;
  // pairs of entries (16-byte accesses; vectors start 256 bytes apart), then an odd last entry
  const int64_t n2 = n >> 1;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n2; i += (int64_t)gridDim.x * blockDim.x) {
    const double2 wi = reinterpret_cast<const double2*>(w)[i];
#pragma unroll
    for (int k = 0; k < kHChunk; ++k)
      if (k < nk) {
        const double2 v = reinterpret_cast<const double2*>(v0 + k * stride)[i];
        acc[k] += v.x * wi.x + v.y * wi.y;
      }
    if (ww) acc[kHChunk] += wi.x * wi.x + wi.y * wi.y;
  }
  if ((n & 1) && blockIdx.x == 0 && threadIdx.x == 0) {
    const double wi = w[n - 1];
#pragma unroll
    for (int k = 0; k < kHChunk; ++k)
      if (k < nk) acc[k] += v0[k * stride + n - 1] * wi;
    if (ww) acc[kHChunk] += wi * wi;
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k <= kHChunk; ++k) {
    double x = acc[k];
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o, 64);
    if (lane == 0) sh[k * (kHThreads / 64) + wv] = x;
  }
  __syncthreads();
  if (threadIdx.x <= kHChunk) {
    const int k = threadIdx.x;
    double x = 0.0;
    for (int i = 0; i < kHThreads / 64; ++i) x += sh[k * (kHThreads / 64) + i];
    if (k < nk) part[(int64_t)(k0 + k) * nbp + blockIdx.x] = x;
    else if (k == kHChunk && ww) part[(int64_t)(kHRows - 1) * nbp + blockIdx.x] = x;
  }
}

// out[k] = sum of the nb partials of row row0 + k (workgroup k, fixed order);
// with sq >= 0, out[sq] = sqrt(out[k_sq]) for the row k_sq = sq - 1.
__global__ __launch_bounds__(kHThreads) void h_mfinal(const double* __restrict__ part, int nbp, int nb, int row0,
                                                      double* __restrict__ out, int sq) {
  __shared__ double sh[kHThreads / 64];
  const double* p = part + (int64_t)(row0 + blockIdx.x) * nbp;
  double v = 0;
  for (int i = threadIdx.x; i < nb; i += blockDim.x) v += p[i];
  v = h_block_sum(v, sh);
  if (threadIdx.x == 0) {
    out[blockIdx.x] = v;
    if (sq >= 0 && (int)blockIdx.x == sq - 1) out[sq] = sqrt(v);
  }
}

// w -= sum_{k < nk} h_k V_{k0+k} in one pass (h on the device); with nrm,
// part[b] = block b's partial sum of the new w . w.
__global__ __launch_bounds__(kHThreads) void h_mupdate(double* __restrict__ w, const double* __restrict__ V,
                                                       int64_t stride, int k0, int nk, const double* __restrict__ h,
                                                       int64_t n, double* __restrict__ part, int nrm) {
  __shared__ double sh[kHThreads / 64];
  double c[kHChunk];
#pragma unroll
  for (int k = 0; k < kHChunk; ++k) c[k] = k < nk ? h[k] : 0.0;
  const double* v0 = V + (int64_t)k0 * stride;
  double q = 0.0;
  const int64_t n2 = n >> 1;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n2; i += (int64_t)gridDim.x * blockDim.x) {
    double2 x = reinterpret_cast<const double2*>(w)[i];
#pragma unroll
    for (int k = 0; k < kHChunk; ++k)
      if (k < nk) {
        const double2 v = reinterpret_cast<const double2*>(v0 + k * stride)[i];
        x.x -= c[k] * v.x;
        x.y -= c[k] * v.y;
      }
    reinterpret_cast<double2*>(w)[i] = x;
    q += x.x * x.x + x.y * x.y;
  }
  if ((n & 1) && blockIdx.x == 0 && threadIdx.x == 0) {
    double x = w[n - 1];
#pragma unroll
    for (int k = 0; k < kHChunk; ++k)
      if (k < nk) x -= c[k] * v0[k * stride + n - 1];
    w[n - 1] = x;
    q += x * x;
  }
  if (nrm) {
    q = h_block_sum(q, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = q;
  }
}

// w = w / (*nrm)
__global__ void h_normalise(double* __restrict__ w, int64_t n, const double* __restrict__ nrm) {
  const double s = 1.0 / *nrm;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    w[i] *= s;
}

__global__ void h_zero(double* __restrict__ x, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    x[i] = 0.0;
}

// r = g (b - x) - r   (residual g b - H x with r = M^{-1} A x on entry)
__global__ void h_residual(double* __restrict__ r, const double* __restrict__ b, const double* __restrict__ x,
                           int64_t n, double g) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    r[i] = g * (b[i] - x[i]) - r[i];
}

struct Coef {
  double y[kHMaxRestart];
};

// x += sum_k y_k V_k   (k < m, V_k = V + k stride)
__global__ void h_update(double* __restrict__ x, const double* __restrict__ V, int64_t stride, int64_t n, int m,
                         const Coef c) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    double s = x[i];
    for (int k = 0; k < m; ++k) s += c.y[k] * V[k * stride + i];
    x[i] = s;
  }
}

size_t up256(size_t b) { return (b + 255) & ~size_t(255); }

struct Gm {
  const dg_mesh* m;
  const double* nut;
  hipStream_t s;
  int64_t n;
  int64_t stride;  // doubles between Krylov vectors
  double* V;       // restart + 1 vectors
  double* sc;      // kHScalars device scalars
  double* part;    // reduction partials
  double gamma;

  double* v(int k) const { return V + k * stride; }
  // y = K x = M^{-1} A x  (y != x)
  int apply_k(const double* x, double* y) {
    int rc = launch_viscous_multiscale(m, nut, x, y, s);
    if (!rc) rc = launch_inverse_mass(m, y, y, s);
    return rc;
  }
  // sc[o + k] = V_k . w for k <= j; with ww also sc[kHSlotW] = w . w
  int proj_dots(const double* w, int j, int o, bool ww) {
    const int nb = h_blocks(n);
    for (int k0 = 0; k0 <= j; k0 += kHChunk) {
      const int nk = std::min(kHChunk, j + 1 - k0);
      hipLaunchKernelGGL(h_mdot, dim3(nb), dim3(kHThreads), 0, s, V, stride, k0, nk, w, n, part, kHMaxParts,
                         (ww && k0 == 0) ? 1 : 0);
    }
    hipLaunchKernelGGL(h_mfinal, dim3(j + 1), dim3(kHThreads), 0, s, part, kHMaxParts, nb, 0, sc + o, -1);
    if (ww)
      hipLaunchKernelGGL(h_mfinal, dim3(1), dim3(kHThreads), 0, s, part, kHMaxParts, nb, kHRows - 1, sc + kHSlotW,
                         -1);
    return check_hip(hipGetLastError(), "helmholtz projections");
  }
  // w -= sum_k sc[o + k] V_k (k <= j); sc[o + j + 1] = ||w||^2, sc[o + j + 2] = ||w||
  int proj_update(double* w, int j, int o) {
    const int nb = h_blocks(n);
    for (int k0 = 0; k0 <= j; k0 += kHChunk) {
      const int nk = std::min(kHChunk, j + 1 - k0);
      hipLaunchKernelGGL(h_mupdate, dim3(nb), dim3(kHThreads), 0, s, w, V, stride, k0, nk, sc + o + k0, n, part,
                         (k0 + nk > j) ? 1 : 0);
    }
    hipLaunchKernelGGL(h_mfinal, dim3(1), dim3(kHThreads), 0, s, part, kHMaxParts, nb, 0, sc + o + j + 1, 1);
    return check_hip(hipGetLastError(), "helmholtz projection update");
  }
  int fetch(double* h, int o, int cnt) {
    return check_hip(hipMemcpyAsync(h, sc + o, sizeof(double) * cnt, hipMemcpyDeviceToHost, s), "read-back");
  }
  // sc[o] = a.b (and sc[o2] = sqrt of it if o2 >= 0)
  int dot(const double* a, const double* b, int o, int o2 = -1) {
    const int nb = h_blocks(n);
    hipLaunchKernelGGL(h_dot, dim3(nb), dim3(kHThreads), 0, s, a, b, n, part);
    hipLaunchKernelGGL(h_final, dim3(1), dim3(kHThreads), 0, s, part, nb, sc + o, o2 >= 0 ? sc + o2 : nullptr);
    return check_hip(hipGetLastError(), "helmholtz reduction");
  }
  int read(double* h, int o, int cnt) {
    if (int rc = check_hip(hipMemcpyAsync(h, sc + o, sizeof(double) * cnt, hipMemcpyDeviceToHost, s), "read-back"))
      return rc;
    return check_hip(hipStreamSynchronize(s), "read-back wait");
  }
};

}  // namespace

int64_t helmholtz_workspace_bytes(const dg_mesh* m, int restart) {
  const size_t vec = up256(sizeof(double) * (size_t)m->n_vel);
  return (int64_t)((size_t)(restart + 1) * vec + up256(sizeof(double) * kHScalars) +
                   up256(sizeof(double) * kHRows * kHMaxParts));
}

int solve_helmholtz(const dg_mesh* m, const double* nut, double gamma, const double* b, double* x, double rtol,
                    int max_iter, int restart, void* ws, size_t ws_bytes, dg_gmres_stats* st, hipStream_t s) {
  const auto t0 = std::chrono::steady_clock::now();
  if (restart < 1 || restart > kHMaxRestart)
    return set_error(DG_ERR_ARG, "GMRES restart length outside [1, 100]");
  if (!(rtol > 0) || max_iter < 1 || !(gamma > 0) || !std::isfinite(gamma))
    return set_error(DG_ERR_ARG, "invalid Helmholtz/GMRES parameters");
  if ((int64_t)ws_bytes < helmholtz_workspace_bytes(m, restart))
    return set_error(DG_ERR_WORKSPACE, "Helmholtz workspace too small");
  if (reinterpret_cast<uintptr_t>(ws) & 255u)  // the Krylov kernels read 16-byte pairs
    return set_error(DG_ERR_ARG, "Helmholtz workspace must be 256-byte aligned");
  Gm G;
  G.m = m;
  G.nut = nut;
  G.s = s;
  G.n = m->n_vel;
  G.stride = (int64_t)(up256(sizeof(double) * (size_t)G.n) / sizeof(double));
  G.V = static_cast<double*>(ws);
  G.sc = G.V + (restart + 1) * G.stride;
  G.part = G.sc + up256(sizeof(double) * kHScalars) / sizeof(double);
  G.gamma = gamma;
  const int SB = kHScalars - 2, SBN = kHScalars - 1;  // ||g b||^2, ||g b||
  int rc;
  // ||gamma b||
  if ((rc = G.dot(b, b, SB, SBN))) return rc;
  double nb;
  if ((rc = G.read(&nb, SBN, 1))) return rc;
  nb *= gamma;
  if (!std::isfinite(nb)) return set_error(DG_ERR_NONFINITE, "non-finite right-hand side");
  dg_gmres_stats stats{};
  if (nb == 0.0) {
    hipLaunchKernelGGL(h_zero, dim3(ew_blocks(G.n)), dim3(256), 0, s, x, G.n);
    if (st) *st = stats;
    return check_hip(hipStreamSynchronize(s), "helmholtz");
  }
  int it = 0, restarts = 0;
  double rel = 1.0;
  std::vector<double> H((size_t)(restart + 1) * restart), cs(restart), sn(restart), g(restart + 1), h(restart + 2),
      h2(restart + 2);
  int reorth = 0;
  bool converged = false;
  while (!converged && it < max_iter) {
    // r = gamma b - H x into V_0, beta = ||r||
    double* r = G.v(0);
    if ((rc = launch_viscous_multiscale(m, nut, x, r, s))) return rc;
    if ((rc = launch_inverse_mass(m, r, r, s))) return rc;
    hipLaunchKernelGGL(h_residual, dim3(ew_blocks(G.n)), dim3(256), 0, s, r, b, x, G.n, gamma);
    if ((rc = G.dot(r, r, 0, 1))) return rc;
    double beta;
    if ((rc = G.read(&beta, 1, 1))) return rc;
    if (!std::isfinite(beta)) return set_error(DG_ERR_NONFINITE, "non-finite residual");
    rel = beta / nb;
    if (rel <= rtol) {
      converged = true;
      break;
    }
    hipLaunchKernelGGL(h_normalise, dim3(ew_blocks(G.n)), dim3(256), 0, s, r, G.n, G.sc + 1);
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = beta;
    int j = 0;
    for (; j < restart && it < max_iter; ++j, ++it) {
      double* w = G.v(j + 1);
      if ((rc = G.apply_k(G.v(j), w))) return rc;
      // classical Gram-Schmidt against V_0 .. V_j, scalars on the device
      if ((rc = G.proj_dots(w, j, 0, true))) return rc;
      if ((rc = G.proj_update(w, j, 0))) return rc;
      double w2 = 0.0;  // ||w||^2 before the projection
      if ((rc = G.fetch(h.data(), 0, j + 3)) || (rc = G.fetch(&w2, kHSlotW, 1))) return rc;
      if ((rc = check_hip(hipStreamSynchronize(s), "read-back wait"))) return rc;
      double hn = h[j + 2];  // ||w|| after the projection
      int slot = j + 2;
      if (!(hn >= std::sqrt(0.5 * w2))) {  // most of w was removed: project once more
        if ((rc = G.proj_dots(w, j, kHPass2, false))) return rc;
        if ((rc = G.proj_update(w, j, kHPass2))) return rc;
        if ((rc = G.read(h2.data(), kHPass2, j + 3))) return rc;
        for (int k = 0; k <= j; ++k) h[k] += h2[k];
        hn = h2[j + 2];
        slot = kHPass2 + j + 2;
        ++reorth;
      }
      if (!std::isfinite(hn)) return set_error(DG_ERR_NONFINITE, "non-finite Arnoldi vector");
      if (hn > 0) hipLaunchKernelGGL(h_normalise, dim3(ew_blocks(G.n)), dim3(256), 0, s, w, G.n, G.sc + slot);
      // Hessenberg column j of H = gamma I + K: h[0..j] (+ gamma on the diagonal), hn; apply the previous
      // rotations, then a new one
      for (int k = 0; k <= j; ++k) H[(size_t)k * restart + j] = h[k];
      H[(size_t)j * restart + j] += gamma;
      H[(size_t)(j + 1) * restart + j] = hn;
      for (int k = 0; k < j; ++k) {
        const double a = H[(size_t)k * restart + j], c = H[(size_t)(k + 1) * restart + j];
        H[(size_t)k * restart + j] = cs[k] * a + sn[k] * c;
        H[(size_t)(k + 1) * restart + j] = -sn[k] * a + cs[k] * c;
      }
      const double a = H[(size_t)j * restart + j], c = H[(size_t)(j + 1) * restart + j];
      const double d = std::hypot(a, c);
      cs[j] = d > 0 ? a / d : 1.0;
      sn[j] = d > 0 ? c / d : 0.0;
      H[(size_t)j * restart + j] = d;
      H[(size_t)(j + 1) * restart + j] = 0.0;
      g[j + 1] = -sn[j] * g[j];
      g[j] = cs[j] * g[j];
      rel = std::fabs(g[j + 1]) / nb;
      if (rel <= rtol || hn == 0.0) {
        ++j;
        ++it;
        converged = true;
        break;
      }
    }
    // x += V y with R y = g (back substitution on the rotated Hessenberg)
    const int kk = j;
    Coef cf{};
    for (int i = kk - 1; i >= 0; --i) {
      double t = g[i];
      for (int k = i + 1; k < kk; ++k) t -= H[(size_t)i * restart + k] * cf.y[k];
      cf.y[i] = t / H[(size_t)i * restart + i];
    }
    hipLaunchKernelGGL(h_update, dim3(ew_blocks(G.n)), dim3(256), 0, s, x, G.V, G.stride, G.n, kk, cf);
    if ((rc = check_hip(hipGetLastError(), "helmholtz update"))) return rc;
    if (!converged) ++restarts;
    else {
      // confirm with the true residual (a restart cycle follows if it is not met)
      double* r = G.v(0);
      if ((rc = launch_viscous_multiscale(m, nut, x, r, s))) return rc;
      if ((rc = launch_inverse_mass(m, r, r, s))) return rc;
      hipLaunchKernelGGL(h_residual, dim3(ew_blocks(G.n)), dim3(256), 0, s, r, b, x, G.n, gamma);
      if ((rc = G.dot(r, r, 0, 1))) return rc;
      double tr;
      if ((rc = G.read(&tr, 1, 1))) return rc;
      rel = tr / nb;
      if (!(rel <= rtol)) {
        converged = false;
        ++restarts;
      }
    }
  }
  stats.iterations = it;
  stats.restarts = restarts;
  stats.reorthogonalised = reorth;
  stats.rel_resid = rel;
  stats.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (st) *st = stats;
  if ((rc = check_hip(hipStreamSynchronize(s), "helmholtz"))) return rc;
  if (!converged) return set_error(DG_ERR_NOT_CONVERGED, "GMRES iteration cap reached");
  return DG_OK;
}

}  // namespace dgwm

using namespace dgwm;

extern "C" {

int64_t dg_helmholtz_workspace_bytes(const dg_mesh* m, const dg_gmres_params* gp) {
  if (!m || !gp) return set_error(DG_ERR_ARG, "mesh/params is NULL");
  if (gp->restart < 1 || gp->restart > kHMaxRestart) return set_error(DG_ERR_ARG, "GMRES restart outside [1, 100]");
  return helmholtz_workspace_bytes(m, gp->restart);
}

int dg_solve_helmholtz(const dg_mesh* m, const double* nut, double gamma0_over_dt, const double* b, double* x,
                       const dg_gmres_params* gp, void* ws, size_t ws_bytes, dg_gmres_stats* st, void* stream) {
  if (!m || !gp || !b || !x || !ws) return set_error(DG_ERR_ARG, "mesh/params/b/x/workspace is NULL");
  if (b == x) return set_error(DG_ERR_ARG, "b and x must not alias");
  if (m->curved) return set_error(DG_ERR_UNSUPPORTED, "the Helmholtz step is built for flat walls only");
  if (m->nenr > 0 && !nut) return set_error(DG_ERR_ARG, "nut is NULL on a mesh with enriched cells");
  return solve_helmholtz(m, nut, gamma0_over_dt, b, x, gp->rtol, gp->max_iter, gp->restart, ws, ws_bytes, st,
                         static_cast<hipStream_t>(stream));
}

}  // extern "C"
