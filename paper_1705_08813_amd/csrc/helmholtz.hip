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
// Arnoldi with modified Gram-Schmidt; every scalar of an Arnoldi step stays
// on the device (the projections are subtracted with their device values) and
// one copy per step brings the new Hessenberg column to the host, where the
// Givens rotations and the least-squares solution live.  Reductions are
// two-stage fixed-grid sums (deterministic).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <vector>

#include "dgwm_internal.h"

namespace dgwm {

namespace {

constexpr int kHThreads = 256;
constexpr int kHMaxParts = 1024;
constexpr int kHScalars = 128;  // device scalars: Hessenberg column (<= restart + 1), norms
constexpr int kHMaxRestart = 100;

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

// w -= (*h) v
__global__ void h_sub_proj(double* __restrict__ w, const double* __restrict__ v, int64_t n,
                           const double* __restrict__ h) {
  const double c = *h;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    w[i] -= c * v[i];
}

// w = w / (*nrm)
__global__ void h_normalise(double* __restrict__ w, int64_t n, const double* __restrict__ nrm) {
  const double s = 1.0 / *nrm;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    w[i] *= s;
}

// y = g x + y  (the operator's gamma x term on top of M^{-1} A x)
__global__ void h_add_scaled(double* __restrict__ y, const double* __restrict__ x, int64_t n, double g) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] += g * x[i];
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
  // y = H x = gamma x + M^{-1} A x  (y != x)
  int apply(const double* x, double* y) {
    int rc = launch_viscous_multiscale(m, nut, x, y, s);
    if (!rc) rc = launch_inverse_mass(m, y, y, s);
    if (rc) return rc;
    hipLaunchKernelGGL(h_add_scaled, dim3(ew_blocks(n)), dim3(256), 0, s, y, x, n, gamma);
    return check_hip(hipGetLastError(), "helmholtz operator");
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
                   up256(sizeof(double) * kHMaxParts));
}

int solve_helmholtz(const dg_mesh* m, const double* nut, double gamma, const double* b, double* x, double rtol,
                    int max_iter, int restart, void* ws, size_t ws_bytes, dg_gmres_stats* st, hipStream_t s) {
  const auto t0 = std::chrono::steady_clock::now();
  if (restart < 1 || restart > kHMaxRestart || restart + 2 > kHScalars)
    return set_error(DG_ERR_ARG, "GMRES restart length outside [1, 100]");
  if (!(rtol > 0) || max_iter < 1 || !(gamma > 0) || !std::isfinite(gamma))
    return set_error(DG_ERR_ARG, "invalid Helmholtz/GMRES parameters");
  if ((int64_t)ws_bytes < helmholtz_workspace_bytes(m, restart))
    return set_error(DG_ERR_WORKSPACE, "Helmholtz workspace too small");
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
  std::vector<double> H((size_t)(restart + 1) * restart), cs(restart), sn(restart), g(restart + 1), h(restart + 2);
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
      if ((rc = G.apply(G.v(j), w))) return rc;
      for (int k = 0; k <= j; ++k) {  // modified Gram-Schmidt, scalars on the device
        if ((rc = G.dot(G.v(k), w, k))) return rc;
        hipLaunchKernelGGL(h_sub_proj, dim3(ew_blocks(G.n)), dim3(256), 0, s, w, G.v(k), G.n, G.sc + k);
      }
      if ((rc = G.dot(w, w, j + 1, j + 2))) return rc;
      if ((rc = G.read(h.data(), 0, j + 3))) return rc;
      const double hn = h[j + 2];  // ||w||
      if (!std::isfinite(hn)) return set_error(DG_ERR_NONFINITE, "non-finite Arnoldi vector");
      if (hn > 0) hipLaunchKernelGGL(h_normalise, dim3(ew_blocks(G.n)), dim3(256), 0, s, w, G.n, G.sc + j + 2);
      // Hessenberg column j: h[0..j], hn; apply the previous rotations, then a new one
      for (int k = 0; k <= j; ++k) H[(size_t)k * restart + j] = h[k];
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
