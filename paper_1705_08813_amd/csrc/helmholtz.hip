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
// with gamma added to its diagonal, which keeps the dominant gamma v_j out of
// the projections.  Orthogonalisation is classical Gram-Schmidt applied twice,
// the second pass delayed into the next Arnoldi step (the DCGS2 scheme of
// Swirydowicz, Langou, Ananthan, Yang and Thomas, 2021, here derived for the
// host-side Hessenberg bookkeeping below): step j applies K to the candidate
// u_j (projected once, not normalised), one read pass over the basis gives the
// projections of both u_j and w = K u_j, and one write pass finishes v_j
// (second projection and normalisation) and forms the once-projected
// candidate u_{j+1}.  The basis vectors are read twice per step instead of
// four (twice-applied classical) or five (modified Gram-Schmidt) times.  Every
// projection coefficient stays on the device (the updates read them there);
// one copy per step brings them to the host, where the Hessenberg matrix, the
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
constexpr int kHMaxRestart = 100;
constexpr int kHChunk = 16;      // basis vectors per pass of the Krylov kernels
// device scalars: projections of the candidate (s, from 0) and of the new
// vector (z, from kHZ), u.u and u.w (kHSlotA, +1), ||gamma b||^2 and ||gamma b||
constexpr int kHZ = 104;
constexpr int kHScalars = 256;
constexpr int kHSlotA = kHScalars - 6;
// rows of reduction partials: s, then z, then u.u and u.w
constexpr int kHRowZ = kHMaxRestart, kHRowA = 2 * kHMaxRestart, kHRows = 2 * kHMaxRestart + 2;

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

// One read pass over nk <= kHChunk basis vectors V_k0 .. V_{k0+nk-1}, the
// candidate u and (hw) the new vector w: block b's partial sums of V_k . u
// (row k0 + k), V_k . w (row kHRowZ + k0 + k) and, with first, u . u and
// u . w (rows kHRowA, kHRowA + 1).
__global__ __launch_bounds__(kHThreads) void h_ddot(const double* __restrict__ V, int64_t stride, int k0, int nk,
                                                    const double* __restrict__ u, const double* __restrict__ w,
                                                    int hw, int64_t n, double* __restrict__ part, int nbp, int first) {
  constexpr int NA = 2 * kHChunk + 2, NW = kHThreads / 64;
  __shared__ double sh[NA * NW];
  double as[kHChunk], az[kHChunk], aa = 0.0, at = 0.0;
#pragma unroll
  for (int k = 0; k < kHChunk; ++k) as[k] = az[k] = 0.0;
  const double* v0 = V + (int64_t)k0 * stride;
  // pairs of entries (16-byte accesses; vectors start 256 bytes apart), then an odd last entry
  const int64_t n2 = n >> 1;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n2; i += (int64_t)gridDim.x * blockDim.x) {
    const double2 ui = reinterpret_cast<const double2*>(u)[i];
    const double2 wi = hw ? reinterpret_cast<const double2*>(w)[i] : double2{0.0, 0.0};
#pragma unroll
    for (int k = 0; k < kHChunk; ++k)
      if (k < nk) {
        const double2 v = reinterpret_cast<const double2*>(v0 + k * stride)[i];
        as[k] += v.x * ui.x + v.y * ui.y;
        az[k] += v.x * wi.x + v.y * wi.y;
      }
    aa += ui.x * ui.x + ui.y * ui.y;
    at += ui.x * wi.x + ui.y * wi.y;
  }
  if ((n & 1) && blockIdx.x == 0 && threadIdx.x == 0) {
    const double ui = u[n - 1], wi = hw ? w[n - 1] : 0.0;
#pragma unroll
    for (int k = 0; k < kHChunk; ++k)
      if (k < nk) {
        const double v = v0[k * stride + n - 1];
        as[k] += v * ui;
        az[k] += v * wi;
      }
    aa += ui * ui;
    at += ui * wi;
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < NA; ++q) {
    double x = q < kHChunk ? as[q] : (q < 2 * kHChunk ? az[q - kHChunk] : (q == 2 * kHChunk ? aa : at));
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o, 64);
    if (lane == 0) sh[q * NW + wv] = x;
  }
  __syncthreads();
  if (threadIdx.x < NA) {
    const int q = threadIdx.x;
    double x = 0.0;
    for (int i = 0; i < NW; ++i) x += sh[q * NW + i];
    int row = -1;
    if (q < kHChunk) row = q < nk ? k0 + q : -1;
    else if (q < 2 * kHChunk) row = (hw && q - kHChunk < nk) ? kHRowZ + k0 + q - kHChunk : -1;
    else if (first) row = kHRowA + (q - 2 * kHChunk);
    if (row >= 0) part[(int64_t)row * nbp + blockIdx.x] = x;
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

// One write pass over a chunk of the basis: u -= sum_k s_k V_{k0+k} and
// (hw) w -= sum_k z_k V_{k0+k}, with s and z on the device; in the last chunk
// also u = u / beta (the finished basis vector v_j) and w = w / beta - g2 u
// (the next candidate; ib = 1 / beta).
__global__ __launch_bounds__(kHThreads) void h_dupdate(double* __restrict__ u, double* __restrict__ w, int hw,
                                                       const double* __restrict__ V, int64_t stride, int k0, int nk,
                                                       const double* __restrict__ sv, const double* __restrict__ zv,
                                                       int64_t n, int last, double ib, double g2) {
  double cs[kHChunk], cz[kHChunk];
#pragma unroll
  for (int k = 0; k < kHChunk; ++k) {
    cs[k] = k < nk ? sv[k0 + k] : 0.0;
    cz[k] = (hw && k < nk) ? zv[k0 + k] : 0.0;
  }
  const double* v0 = V + (int64_t)k0 * stride;
  const int64_t n2 = n >> 1;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n2; i += (int64_t)gridDim.x * blockDim.x) {
    double2 a = reinterpret_cast<const double2*>(u)[i];
    double2 c = hw ? reinterpret_cast<const double2*>(w)[i] : double2{0.0, 0.0};
#pragma unroll
    for (int k = 0; k < kHChunk; ++k)
      if (k < nk) {
        const double2 v = reinterpret_cast<const double2*>(v0 + k * stride)[i];
        a.x -= cs[k] * v.x;
        a.y -= cs[k] * v.y;
        c.x -= cz[k] * v.x;
        c.y -= cz[k] * v.y;
      }
    if (last) {
      a.x *= ib;
      a.y *= ib;
      c.x = c.x * ib - g2 * a.x;
      c.y = c.y * ib - g2 * a.y;
    }
    reinterpret_cast<double2*>(u)[i] = a;
    if (hw) reinterpret_cast<double2*>(w)[i] = c;
  }
  if ((n & 1) && blockIdx.x == 0 && threadIdx.x == 0) {
    double a = u[n - 1], c = hw ? w[n - 1] : 0.0;
#pragma unroll
    for (int k = 0; k < kHChunk; ++k)
      if (k < nk) {
        const double v = v0[k * stride + n - 1];
        a -= cs[k] * v;
        c -= cz[k] * v;
      }
    if (last) {
      a *= ib;
      c = c * ib - g2 * a;
    }
    u[n - 1] = a;
    if (hw) w[n - 1] = c;
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
  const double* nut;     // multiscale viscous operator: nu_t of the enriched points
  const double* tau_d;   // div-div operator (when not null): tau_D per cell
  hipStream_t s;
  int64_t n;
  int64_t stride;  // doubles between Krylov vectors
  double* V;       // restart + 1 vectors
  double* sc;      // kHScalars device scalars
  double* part;    // reduction partials
  double gamma;

  double* v(int k) const { return V + k * stride; }
  // y = K x = M^{-1} A x  (y != x), A the multiscale viscous operator or, with tau_d, the div-div penalty
  int apply_k(const double* x, double* y) {
    int rc = tau_d ? launch_divdiv(m, false, x, tau_d, 0.0, y, s) : launch_viscous_multiscale(m, nut, x, y, s);
    if (!rc) rc = launch_inverse_mass(m, y, y, s);
    return rc;
  }
  // projections of the candidate u = V_j on V_0 .. V_{j-1} into sc[0 ..] and, with w, of w into sc[kHZ ..];
  // u.u and u.w into sc[kHSlotA], sc[kHSlotA + 1]
  int ddots(int j, const double* w) {
    const int nb = h_blocks(n);
    const double* u = v(j);
    for (int k0 = 0; k0 == 0 || k0 < j; k0 += kHChunk) {
      const int nk = std::min(kHChunk, j - k0);
      hipLaunchKernelGGL(h_ddot, dim3(nb), dim3(kHThreads), 0, s, V, stride, k0, nk, u, w, w ? 1 : 0, n, part,
                         kHMaxParts, k0 == 0 ? 1 : 0);
    }
    if (j > 0) {
      hipLaunchKernelGGL(h_mfinal, dim3(j), dim3(kHThreads), 0, s, part, kHMaxParts, nb, 0, sc, -1);
      if (w) hipLaunchKernelGGL(h_mfinal, dim3(j), dim3(kHThreads), 0, s, part, kHMaxParts, nb, kHRowZ, sc + kHZ, -1);
    }
    hipLaunchKernelGGL(h_mfinal, dim3(2), dim3(kHThreads), 0, s, part, kHMaxParts, nb, kHRowA, sc + kHSlotA, -1);
    return check_hip(hipGetLastError(), "helmholtz projections");
  }
  // V_j = (V_j - sum_k s_k V_k) / beta and V_{j+1} = (V_{j+1} - sum_k z_k V_k) / beta - g2 V_j (k < j)
  int dupdate(int j, bool hw, double ib, double g2) {
    double* u = v(j);
    double* w = hw ? v(j + 1) : nullptr;
    for (int k0 = 0; k0 == 0 || k0 < j; k0 += kHChunk) {
      const int nk = std::min(kHChunk, j - k0);
      hipLaunchKernelGGL(h_dupdate, dim3(h_blocks(n)), dim3(kHThreads), 0, s, u, w, hw ? 1 : 0, V, stride, k0, nk,
                         sc, sc + kHZ, n, (k0 + kHChunk >= j) ? 1 : 0, ib, g2);
    }
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

// gamma x + M^{-1} A x = gamma b, A the multiscale viscous operator (tau_d null) or the div-div penalty
static int solve_shifted(const dg_mesh* m, const double* nut, const double* tau_d, double gamma, const double* b,
                         double* x, double rtol, int max_iter, int restart, void* ws, size_t ws_bytes,
                         dg_gmres_stats* st, hipStream_t s) {
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
  G.tau_d = tau_d;
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
  // HK: Hessenberg matrix of K (unrotated, row-major with row length restart); R: that of H = gamma I + K after
  // the Givens rotations; g: the rotated right-hand side
  const size_t ld = (size_t)restart;
  std::vector<double> HK((restart + 1) * ld), R((restart + 1) * ld), cs(restart), sn(restart), g(restart + 1),
      sv(restart + 1), zv(restart + 1), y(restart + 1);
  bool converged = false;
  while (!converged && it < max_iter) {
    // r = gamma b - H x into V_0, beta = ||r||
    double* r = G.v(0);
    if ((rc = G.apply_k(x, r))) return rc;
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
    std::fill(HK.begin(), HK.end(), 0.0);
    g[0] = beta;
    // Step j: V_0 .. V_{j-1} are finished basis vectors, V_j holds the candidate u_j (projected once, not
    // normalised; for j = 0 the finished v_0).  Columns 0 .. j-2 of HK are final, column j-1 still lacks the
    // second projection of u_j and its subdiagonal ||u_j - V s||.
    int j = 0, dim = 0;
    for (;; ++j) {
      const bool more = j < restart && it < max_iter;  // another Arnoldi step follows this one
      double* w = more ? G.v(j + 1) : nullptr;
      if (more && (rc = G.apply_k(G.v(j), w))) return rc;
      if ((rc = G.ddots(j, w))) return rc;
      double au[2] = {0.0, 0.0};  // u.u, u.w
      if ((j > 0 && (rc = G.fetch(sv.data(), 0, j))) || (more && j > 0 && (rc = G.fetch(zv.data(), kHZ, j))) ||
          (rc = G.fetch(au, kHSlotA, 2)))
        return rc;
      if ((rc = check_hip(hipStreamSynchronize(s), "read-back wait"))) return rc;
      double ss = 0.0, sz = 0.0;
      for (int k = 0; k < j; ++k) {
        ss += sv[k] * sv[k];
        sz += sv[k] * zv[k];
      }
      // the candidate's norm after its second projection (Pythagoras: s is small against u)
      const double b2 = j > 0 ? au[0] - ss : 1.0;
      if (!std::isfinite(b2) || !std::isfinite(au[1])) return set_error(DG_ERR_NONFINITE, "non-finite Arnoldi vector");
      const double bj = b2 > 0.0 ? std::sqrt(b2) : 0.0;
      if (j > 0) {
        // finish column j-1: K v_{j-1} = sum_k (HK[k][j-1] + s_k) v_k + beta_j v_j
        for (int k = 0; k < j; ++k) HK[k * ld + j - 1] += sv[k];
        HK[j * ld + j - 1] = bj;
        // its column of H = gamma I + K, rotated
        const int c = j - 1;
        for (int k = 0; k <= j; ++k) R[k * ld + c] = HK[k * ld + c];
        R[c * ld + c] += gamma;
        for (int k = 0; k < c; ++k) {
          const double a = R[k * ld + c], d = R[(k + 1) * ld + c];
          R[k * ld + c] = cs[k] * a + sn[k] * d;
          R[(k + 1) * ld + c] = -sn[k] * a + cs[k] * d;
        }
        const double a = R[c * ld + c], d = R[(c + 1) * ld + c];
        const double hyp = std::hypot(a, d);
        cs[c] = hyp > 0 ? a / hyp : 1.0;
        sn[c] = hyp > 0 ? d / hyp : 0.0;
        R[c * ld + c] = hyp;
        R[(c + 1) * ld + c] = 0.0;
        g[c + 1] = -sn[c] * g[c];
        g[c] = cs[c] * g[c];
        rel = std::fabs(g[c + 1]) / nb;
        dim = j;
        if (rel <= rtol || bj == 0.0) {
          converged = true;
          break;
        }
      }
      if (!more) break;
      // column j: with v_j = (u_j - V s) / beta_j, K v_j = (w - K V s) / beta_j and K V s = V_{j+1} HK s, so
      // HK[k][j] = v_k . K v_j = (z_k - (HK s)_k) / beta_j (k < j), HK[j][j] = (gj - (HK s)_j) / beta_j with
      // gj = v_j . w = (u.w - s.z) / beta_j, and u_{j+1} = (w - V z) / beta_j - (gj / beta_j) v_j
      const double gj = (au[1] - sz) / bj;
      for (int k = 0; k <= j; ++k) {
        double t = 0.0;
        for (int l = 0; l < j; ++l) t += HK[k * ld + l] * sv[l];
        y[k] = t;
      }
      for (int k = 0; k < j; ++k) HK[k * ld + j] = (zv[k] - y[k]) / bj;
      HK[j * ld + j] = (gj - y[j]) / bj;
      if ((rc = G.dupdate(j, true, 1.0 / bj, gj / bj))) return rc;
      ++it;
    }
    // x += V y with R y = g (back substitution on the rotated Hessenberg matrix)
    const int kk = dim;
    Coef cf{};
    for (int i = kk - 1; i >= 0; --i) {
      double t = g[i];
      for (int k = i + 1; k < kk; ++k) t -= R[(size_t)i * ld + k] * cf.y[k];
      cf.y[i] = t / R[(size_t)i * ld + i];
    }
    hipLaunchKernelGGL(h_update, dim3(ew_blocks(G.n)), dim3(256), 0, s, x, G.V, G.stride, G.n, kk, cf);
    if ((rc = check_hip(hipGetLastError(), "helmholtz update"))) return rc;
    if (!converged) ++restarts;
    else {
      // confirm with the true residual (a restart cycle follows if it is not met)
      double* r = G.v(0);
      if ((rc = G.apply_k(x, r))) return rc;
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

int solve_helmholtz(const dg_mesh* m, const double* nut, double gamma, const double* b, double* x, double rtol,
                    int max_iter, int restart, void* ws, size_t ws_bytes, dg_gmres_stats* st, hipStream_t s) {
  return solve_shifted(m, nut, nullptr, gamma, b, x, rtol, max_iter, restart, ws, ws_bytes, st, s);
}

// The projection step (M + D) x = M b' as x + M^{-1} D x = b' (b' = u_hat - s M^{-1} g): block diagonal, one
// GMRES over all cells (used for degree-1 enrichment weights, whose enriched cells have no direct solve here).
int solve_projection_gmres(const dg_mesh* m, const double* tau_d, const double* b, double* x, double rtol,
                           int max_iter, int restart, void* ws, size_t ws_bytes, dg_gmres_stats* st, hipStream_t s) {
  return solve_shifted(m, nullptr, tau_d, 1.0, b, x, rtol, max_iter, restart, ws, ws_bytes, st, s);
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
