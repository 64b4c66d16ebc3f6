// Poisson solve for the singular SIP operator (pressure step of the paper's
// dual-splitting scheme, Sec. 4.1 eq. poisson, with the operator of Sec. 4.2).
//
// Outer loop: flexible preconditioned conjugate gradients in FP64 (residuals,
// norms, dot products and the solution always FP64), with the true residual
// b - A x recomputed (residual replacement) every few iterations and before
// accepting convergence.  Preconditioner:
//   multigrid: one V-cycle over the mesh's nested levels (the paper's solver
//              is multigrid-preconditioned, Sec. 4.4), Chebyshev-Jacobi
//              smoothing (degree m on the finest level, a separate, usually
//              lower degree below it), restriction/prolongation of
//              kern_mg.hip, dense pseudo-inverse on the coarsest level;
//   otherwise: Chebyshev polynomial of degree m in D^{-1} A on
//              [lmax/30, 1.1 lmax], optionally wrapped in FP32 CG iterations.
// mixed = 1 runs the preconditioner in FP32 on the normalised residual.
// lmax of each level from 20 Lanczos steps (Jacobi-preconditioned CG
// coefficients kept on the device), cached in the mesh handle.
// Every reduction is a fixed-grid two-stage FP64 sum: deterministic.
// The null space (constants) is handled by projecting b and x to zero mean.
#include <algorithm>
#include <chrono>
#include <functional>
#include <mutex>
#include <string>
#include <cmath>
#include <cstring>
#include <type_traits>
#include <vector>

#include "batch.h"

namespace dgwm {

namespace {

constexpr int kRedBlocks = 2048;  // most partial sums of one reduction (workspace sizing)
constexpr double kSmoothRange = 20.0;  // multigrid smoother interval [lmax / 20, 1.1 lmax]
constexpr int kRedThreads = 256;

// Workgroups of a reduction over n entries: a function of n only, so that a
// vector's partial sums, and hence its result, do not depend on the launch
// (single solve or batch); about one entry per thread for small vectors.
inline int red_blocks(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>((n + 511) / 512, 1024)); }

__device__ __forceinline__ double block_reduce(double v, double* sh) {
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

template <typename TA, typename TB>
__global__ __launch_bounds__(kRedThreads) void k_dot(const TA* __restrict__ a, const TB* __restrict__ b, int64_t n,
                                                     double* __restrict__ part) {
  __shared__ double sh[kRedThreads / 64];
  double v = 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    v += (double)a[i] * (double)b[i];
  v = block_reduce(v, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = v;
}

// a.b1 and a.b2 in one pass (partials of the second at part + gridDim.x)
__global__ __launch_bounds__(kRedThreads) void k_dot2(const double* __restrict__ a, const double* __restrict__ b1,
                                                      const double* __restrict__ b2, int64_t n,
                                                      double* __restrict__ part) {
  __shared__ double sh[kRedThreads / 64];
  double v1 = 0, v2 = 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double ai = a[i];
    v1 += ai * b1[i];
    v2 += ai * b2[i];
  }
  v1 = block_reduce(v1, sh);
  __syncthreads();
  v2 = block_reduce(v2, sh);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = v1;
    part[gridDim.x + blockIdx.x] = v2;
  }
}

template <typename T>
__global__ __launch_bounds__(kRedThreads) void k_sum(const T* __restrict__ a, int64_t n, double* __restrict__ part) {
  __shared__ double sh[kRedThreads / 64];
  double v = 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    v += (double)a[i];
  v = block_reduce(v, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = v;
}

// *out = sum of the nb partials at part, *out2 (if not null) of the nb at
// part + nb (one block, fixed order).
__global__ __launch_bounds__(kRedThreads) void k_final(const double* __restrict__ part, int nb,
                                                       double* __restrict__ out, double* __restrict__ out2) {
  __shared__ double sh[kRedThreads / 64];
  double v = 0;
  for (int i = threadIdx.x; i < nb; i += blockDim.x) v += part[i];
  v = block_reduce(v, sh);
  if (threadIdx.x == 0) *out = v;
  if (!out2) return;
  __syncthreads();
  v = 0;
  for (int i = threadIdx.x; i < nb; i += blockDim.x) v += part[nb + i];
  v = block_reduce(v, sh);
  if (threadIdx.x == 0) *out2 = v;
}

template <typename T>
__global__ void k_sub_mean(T* __restrict__ a, int64_t n, const double* __restrict__ sum) {
  const double mean = *sum / (double)n;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    a[i] = (T)((double)a[i] - mean);
}

// y = b - mean(b)
__global__ void k_copy_sub_mean(double* __restrict__ y, const double* __restrict__ b, int64_t n,
                                const double* __restrict__ sum) {
  const double mean = *sum / (double)n;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = b[i] - mean;
}

// r = b - Ax
__global__ void k_resid(double* __restrict__ r, const double* __restrict__ b, const double* __restrict__ ax, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    r[i] = b[i] - ax[i];
}

// x += alpha p, r -= alpha q with alpha = num/den (device scalars); partial
// sums of r^2.  With r32 != nullptr the new residual is also written in FP32,
// divided by sqrt(*rr_prev) (the previous residual norm, which keeps the FP32
// copy near unit size); that divisor is stored in *scl for the way back.
template <typename T>
__global__ __launch_bounds__(kRedThreads) void k_update_xr(T* __restrict__ x, T* __restrict__ r,
                                                          const T* __restrict__ p, const T* __restrict__ q, int64_t n,
                                                          const double* __restrict__ num,
                                                          const double* __restrict__ den, double* __restrict__ part,
                                                          float* __restrict__ r32 = nullptr,
                                                          const double* __restrict__ rr_prev = nullptr,
                                                          double* __restrict__ scl = nullptr) {
  __shared__ double sh[kRedThreads / 64];
  const T alpha = (T)(*num / *den);
  const double nrm = r32 ? sqrt(*rr_prev) : 1.0, inv = 1.0 / nrm;
  if (r32 && blockIdx.x == 0 && threadIdx.x == 0) *scl = nrm;
  double v = 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    x[i] += alpha * p[i];
    const T ri = r[i] - alpha * q[i];
    r[i] = ri;
    if (r32) r32[i] = (float)(ri * inv);
    v += (double)ri * (double)ri;
  }
  v = block_reduce(v, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = v;
}

// p = z + beta p, beta = (num - sub) / den
template <typename T>
__global__ void k_update_p(T* __restrict__ p, const T* __restrict__ z, int64_t n, const double* __restrict__ num,
                           const double* __restrict__ sub, const double* __restrict__ den) {
  const double nb = *num - (sub ? *sub : 0.0);
  const T beta = (T)(nb / *den);
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = z[i] + beta * p[i];
}

// Chebyshev first step: d = c Dinv r, z = d
template <typename T>
__global__ void k_cheb_first(T* __restrict__ z, T* __restrict__ d, const T* __restrict__ r,
                             const T* __restrict__ dinv, int64_t n, T c) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const T v = c * dinv[i] * r[i];
    d[i] = v;
    z[i] = v;
  }
}

// Chebyshev step: d = c1 d + c2 Dinv (r - Az), z += d
template <typename T>
__global__ void k_cheb_step(T* __restrict__ z, T* __restrict__ d, const T* __restrict__ r, const T* __restrict__ az,
                            const T* __restrict__ dinv, int64_t n, T c1, T c2) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const T v = c1 * d[i] + c2 * dinv[i] * (r[i] - az[i]);
    d[i] = v;
    z[i] += v;
  }
}

// out32 = r / sqrt(rr); the divisor is stored in *scl
__global__ void k_to_f32(float* __restrict__ out, const double* __restrict__ r, int64_t n,
                         const double* __restrict__ rr, double* __restrict__ scl) {
  const double nrm = sqrt(*rr), s = 1.0 / nrm;
  if (blockIdx.x == 0 && threadIdx.x == 0) *scl = nrm;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    out[i] = (float)(r[i] * s);
}

// z = scl * x32
__global__ void k_from_f32(double* __restrict__ z, const float* __restrict__ x, int64_t n,
                           const double* __restrict__ scl) {
  const double s = *scl;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    z[i] = s * (double)x[i];
}

// z = scl * x32 together with the partial sums of r.z and (zold != nullptr)
// r.zold (second set at part + gridDim.x)
__global__ __launch_bounds__(kRedThreads) void k_from_f32_dot2(double* __restrict__ z, const float* __restrict__ x,
                                                               const double* __restrict__ scl,
                                                               const double* __restrict__ r,
                                                               const double* __restrict__ zold, int64_t n,
                                                               double* __restrict__ part) {
  __shared__ double sh[kRedThreads / 64];
  const double s = *scl;
  double v1 = 0, v2 = 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double zi = s * (double)x[i], ri = r[i];
    z[i] = zi;
    v1 += ri * zi;
    if (zold) v2 += ri * zold[i];
  }
  v1 = block_reduce(v1, sh);
  __syncthreads();
  v2 = block_reduce(v2, sh);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = v1;
    part[gridDim.x + blockIdx.x] = v2;
  }
}

template <typename T>
__global__ void k_recip(T* __restrict__ out, const double* __restrict__ d, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    out[i] = (T)(1.0 / d[i]);
}

template <typename T>
__global__ void k_fill(T* __restrict__ a, int64_t n, T v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    a[i] = v;
}

template <typename T>
__global__ void k_copy(T* __restrict__ a, const T* __restrict__ b, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    a[i] = b[i];
}

// deterministic pseudo-random start vector in [-1, 1] (integer hash of the index)
__global__ void k_hash_fill(double* __restrict__ a, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    uint64_t z = (uint64_t)i + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    a[i] = (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
  }
}

// largest eigenvalue of a symmetric tridiagonal matrix (Sturm bisection)
double tridiag_max_eig(const double* a, const double* b, int n) {
  double lo = 1e300, hi = -1e300;
  for (int i = 0; i < n; ++i) {
    const double r = (i > 0 ? std::fabs(b[i - 1]) : 0) + (i + 1 < n ? std::fabs(b[i]) : 0);
    lo = std::fmin(lo, a[i] - r);
    hi = std::fmax(hi, a[i] + r);
  }
  auto count_below = [&](double x) {
    int c = 0;
    double q = a[0] - x;
    if (q < 0) ++c;
    for (int i = 1; i < n; ++i) {
      if (q == 0) q = 1e-300;
      q = a[i] - x - b[i - 1] * b[i - 1] / q;
      if (q < 0) ++c;
    }
    return c;
  };
  for (int it = 0; it < 200 && hi - lo > 1e-14 * std::fabs(hi); ++it) {
    const double mid = 0.5 * (lo + hi);
    if (count_below(mid) >= n) hi = mid; else lo = mid;
  }
  return hi;
}

struct Solver {
  const dg_mesh* m;
  hipStream_t s;
  int64_t n;
  unsigned grid;
  double *bp, *r, *z, *zold, *p, *q, *d64, *t64, *dinv, *sc, *part;
  float *r32, *z32, *d32, *t32, *x32, *rr32, *pp32, *qq32, *dinv32;
  int applies64 = 0, applies32 = 0, inner_total = 0;
  int nred = 1;  // partials of the last reduction launched

  // workgroups of a reduction over nn entries (remembered for red_final)
  unsigned red(int64_t nn) {
    nred = red_blocks(nn);
    return (unsigned)nred;
  }
  int red_final(double* out, double* out2 = nullptr) {
    hipLaunchKernelGGL(k_final, dim3(1), dim3(kRedThreads), 0, s, part, nred, out, out2);
    return check_hip(hipGetLastError(), "reduce");
  }
  // a.b1 -> out1, a.b2 -> out2 in one pass over a
  int dot2(const double* a, const double* b1, const double* b2, double* out1, double* out2) {
    hipLaunchKernelGGL(k_dot2, dim3(red(n)), dim3(kRedThreads), 0, s, a, b1, b2, n, part);
    return red_final(out1, out2);
  }
  template <typename TA, typename TB>
  int dot(const TA* a, const TB* b, double* out, int64_t nn = -1) {
    if (nn < 0) nn = n;
    hipLaunchKernelGGL((k_dot<TA, TB>), dim3(red(nn)), dim3(kRedThreads), 0, s, a, b, nn, part);
    return red_final(out);
  }
  template <typename T>
  int project(T* a, double* sum, int64_t nn = -1) {
    if (nn < 0) nn = n;
    hipLaunchKernelGGL((k_sum<T>), dim3(red(nn)), dim3(kRedThreads), 0, s, a, nn, part);
    int rc = red_final(sum);
    if (rc) return rc;
    hipLaunchKernelGGL((k_sub_mean<T>), dim3(grid_of(nn)), dim3(256), 0, s, a, nn, sum);
    return check_hip(hipGetLastError(), "sub mean");
  }
  int A64(const double* x, double* y) {
    ++applies64;
    return launch_poisson(m, DG_F64, x, y, s);
  }
  int A32(const float* x, float* y) {
    ++applies32;
    return launch_poisson(m, DG_F32, x, y, s);
  }
  // ---- multigrid (levels 1.. of the mesh hierarchy) ----
  struct Lv {
    char* x;
    char* b;
    char* r;
    char* t;
    double* dinv64;
    float* dinv32;
    int64_t n;
  };
  Lv lv[kMaxLevels];
  int nlev = 0;
  static unsigned grid_of(int64_t n) { return (unsigned)std::min<int64_t>((n + 255) / 256, 2048); }
  template <typename T>
  int Alev(int l, const T* x, T* y) {
    if (l == 0) {
      if (sizeof(T) == 8) ++applies64; else ++applies32;
    }
    return launch_poisson_level(m, l, sizeof(T) == 8 ? DG_F64 : DG_F32, x, y, s);
  }
  template <typename T>
  const T* dinv_of(int l) {
    if (sizeof(T) == 8) return reinterpret_cast<const T*>(l == 0 ? dinv : lv[l].dinv64);
    return reinterpret_cast<const T*>(l == 0 ? dinv32 : lv[l].dinv32);
  }
  int64_t n_of(int l) const { return l == 0 ? n : lv[l].n; }
  // z = Cheb_m(D^{-1} A_l) D^{-1} r from a zero start (m - 1 operator
  // applications, each fused with its recurrence step).  The iterates
  // ping-pong between z and t, each step overwriting the iterate before the
  // previous one (which the kernel reads first), arranged to end in z.
  template <typename T>
  int cheb_l(int l, T* zz, const T* rr, T* tt, int deg, double lmin, double lmax) {
    const int64_t nn = n_of(l);
    const unsigned g = grid_of(nn);
    const T* di = dinv_of<T>(l);
    const double theta = 0.5 * (lmax + lmin), delta = 0.5 * (lmax - lmin), sigma = theta / delta;
    double rho = 1.0 / sigma;
    T* cur = ((deg - 1) % 2) ? tt : zz;
    T* oth = cur == zz ? tt : zz;
    if (deg == 1)  // (the second output is scratch)
      hipLaunchKernelGGL((k_cheb_first<T>), dim3(g), dim3(256), 0, s, cur, oth, rr, di, nn, (T)(1.0 / theta));
    for (int k = 1; k < deg; ++k) {
      const double rho_new = 1.0 / (2.0 * sigma - rho);
      if (l == 0) {
        if (sizeof(T) == 8) ++applies64; else ++applies32;
      }
      const T c1 = (T)(rho_new * rho), c2 = (T)(2.0 * rho_new / delta);
      // the first application forms the first iterate D^{-1} r / theta itself
      // and stores it in cur, where the second one finds it
      int rc = k == 1 ? launch_poisson_cheb_first<T>(m, l, (T)(1.0 / theta), oth, cur, rr, di, c1, c2, s)
                      : launch_poisson_cheb<T>(m, l, cur, oth, rr, di, c1, c2, s);
      if (rc) return rc;
      std::swap(cur, oth);
      rho = rho_new;
    }
    return check_hip(hipGetLastError(), "chebyshev");
  }
  // the same polynomial continued from the current iterate, which the
  // caller has put in t for an odd step count and in x for an even one, so
  // that the m fused operator applications end in x
  template <typename T>
  int cheb_from(int l, T* xx, const T* bb, T* tt, int deg, double lmin, double lmax) {
    const T* di = dinv_of<T>(l);
    const double theta = 0.5 * (lmax + lmin), delta = 0.5 * (lmax - lmin), sigma = theta / delta;
    double rho = 1.0 / sigma;
    T* cur = (deg % 2) ? tt : xx;
    T* oth = cur == xx ? tt : xx;
    for (int k = 0; k < deg; ++k) {
      T c1 = 0, c2 = (T)(1.0 / theta);
      if (k > 0) {
        const double rho_new = 1.0 / (2.0 * sigma - rho);
        c1 = (T)(rho_new * rho);
        c2 = (T)(2.0 * rho_new / delta);
        rho = rho_new;
      }
      if (l == 0) {
        if (sizeof(T) == 8) ++applies64; else ++applies32;
      }
      int rc = launch_poisson_cheb<T>(m, l, cur, oth, bb, di, c1, c2, s);
      if (rc) return rc;
      std::swap(cur, oth);
    }
    return check_hip(hipGetLastError(), "chebyshev");
  }
  // x = V-cycle(l) b: Chebyshev-Jacobi pre-smoothing, restricted residual,
  // coarse correction, post-smoothing; the coarsest level is solved with the
  // dense pseudo-inverse (or smoothed with a long polynomial).
  template <typename T>
  int vcycle(int l, T* x, const T* b, T* r, T* t, int deg0, int degc) {
    const int deg = l == 0 ? deg0 : degc;  // smoothing degree on this level
    const dg_mesh* mm = m;
    const int L = nlev - 1;
    const int64_t nn = n_of(l);
    const double lam = mm->mg[l].lam;
    const dg_prec prec = sizeof(T) == 8 ? DG_F64 : DG_F32;
    int rc;
    if (l == L) {
      if (mm->coarse_inv)
        return launch_dense_apply(nn, prec, sizeof(T) == 8 ? (const void*)mm->coarse_inv : (const void*)mm->coarse_inv32,
                                  b, x, s);
      return cheb_l<T>(l, x, b, t, 4 * deg0, lam / 200.0, 1.1 * lam);
    }
    const double lmin = lam / kSmoothRange, lmax = 1.1 * lam;
    if ((rc = cheb_l<T>(l, x, b, t, deg, lmin, lmax))) return rc;
    if (l == 0) {
      if (sizeof(T) == 8) ++applies64; else ++applies32;
    }
    if ((rc = launch_poisson_resid<T>(mm, l, x, b, r, s))) return rc;
    Lv& c = lv[l + 1];
    T* xc = reinterpret_cast<T*>(c.x);
    T* bc = reinterpret_cast<T*>(c.b);
    if ((rc = launch_mg_restrict(mm, l, prec, r, bc, s))) return rc;
    if ((rc = vcycle<T>(l + 1, xc, bc, reinterpret_cast<T*>(c.r), reinterpret_cast<T*>(c.t), deg0, degc)))
      return rc;
    // coarse correction into the buffer the post-smoothing starts from
    if ((rc = launch_mg_prolong_add(mm, l, prec, xc, x, (deg % 2) ? t : x, s))) return rc;
    return cheb_from<T>(l, x, b, t, deg, lmin, lmax);
  }
  // Lanczos estimate of lmax(D^{-1} A_l) (20 Jacobi-PCG steps in FP64 on
  // level l, using the level-0 work vectors, which are at least as long)
  int lanczos(int l, double* out);

  // blocking read of one device scalar (NaN if the copy fails)
  double host(const double* dev) {
    double h = 0;
    if (hipMemcpyAsync(&h, dev, sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess) return NAN;
    if (hipStreamSynchronize(s) != hipSuccess) return NAN;
    return h;
  }
  // z = Cheb_m(D^{-1} A) D^{-1} r in precision T, using temporaries d, t
  template <typename T>
  int cheb(T* zz, const T* rr, T* dd, T* tt, const T* di, int deg, double lmin, double lmax) {
    const double theta = 0.5 * (lmax + lmin), delta = 0.5 * (lmax - lmin), sigma = theta / delta;
    double rho = 1.0 / sigma;
    hipLaunchKernelGGL((k_cheb_first<T>), dim3(grid), dim3(256), 0, s, zz, dd, rr, di, n, (T)(1.0 / theta));
    for (int k = 1; k < deg; ++k) {
      int rc = (sizeof(T) == 8) ? A64((const double*)zz, (double*)tt) : A32((const float*)zz, (float*)tt);
      if (rc) return rc;
      const double rho_new = 1.0 / (2.0 * sigma - rho);
      hipLaunchKernelGGL((k_cheb_step<T>), dim3(grid), dim3(256), 0, s, zz, dd, rr, tt, di, n,
                         (T)(rho_new * rho), (T)(2.0 * rho_new / delta));
      rho = rho_new;
    }
    return check_hip(hipGetLastError(), "chebyshev");
  }
};

int Solver::lanczos(int l, double* out) {
  // 20 Jacobi-PCG steps with every scalar kept on the device (no host
  // synchronisation inside the loop); the CG coefficients come back in one
  // copy and give the Lanczos tridiagonal.  A breakdown (exact convergence on
  // a tiny level) only truncates the valid prefix.
  constexpr int K = 20;
  const int64_t nn = n_of(l);
  const unsigned g = grid_of(nn);
  const double* di = dinv_of<double>(l);
  double* RZ = sc + 20;  // sc[20..39]
  double* PQ = sc + 40;  // sc[40..59]
  hipLaunchKernelGGL(k_hash_fill, dim3(g), dim3(256), 0, s, r, nn);
  int rc = project(r, sc + 16, nn);
  if (rc) return rc;
  hipLaunchKernelGGL((k_fill<double>), dim3(g), dim3(256), 0, s, t64, nn, 0.0);
  for (int k = 0; k < K; ++k) {
    hipLaunchKernelGGL((k_cheb_first<double>), dim3(g), dim3(256), 0, s, z, d64, r, di, nn, 1.0);
    if ((rc = dot(r, z, RZ + k, nn))) return rc;
    if (k == 0)
      hipLaunchKernelGGL((k_copy<double>), dim3(g), dim3(256), 0, s, p, z, nn);
    else
      hipLaunchKernelGGL((k_update_p<double>), dim3(g), dim3(256), 0, s, p, z, nn, RZ + k, (const double*)nullptr,
                         RZ + k - 1);
    if ((rc = launch_poisson_level(m, l, DG_F64, p, q, s))) return rc;
    if ((rc = dot(p, q, PQ + k, nn))) return rc;
    hipLaunchKernelGGL((k_update_xr<double>), dim3(red(nn)), dim3(kRedThreads), 0, s, t64, r, p, q, nn, RZ + k,
                       PQ + k, part, (float*)nullptr, (const double*)nullptr, (double*)nullptr);
  }
  double h[2 * K];
  if ((rc = check_hip(hipMemcpyAsync(h, RZ, sizeof(double) * 2 * K, hipMemcpyDeviceToHost, s), "lanczos copy")))
    return rc;
  if ((rc = check_hip(hipStreamSynchronize(s), "lanczos"))) return rc;
  double al[K], be[K], diag[K], off[K];
  int kk = 0;
  for (int k = 0; k < K; ++k) {
    const double rz = h[k], pq = h[K + k];
    if (!(rz > 0) || !(pq > 0) || !std::isfinite(rz) || !std::isfinite(pq)) break;
    if (k > 0) be[k - 1] = rz / h[k - 1];
    al[k] = rz / pq;
    kk = k + 1;
  }
  if (kk < 1) return set_error(DG_ERR_NONFINITE, "eigenvalue estimate failed");
  for (int j = 0; j < kk; ++j) {
    diag[j] = 1.0 / al[j] + (j > 0 ? be[j - 1] / al[j - 1] : 0.0);
    if (j + 1 < kk) off[j] = std::sqrt(be[j]) / al[j];
  }
  *out = tridiag_max_eig(diag, off, kk);
  return DG_OK;
}

}  // namespace
}  // namespace dgwm

using namespace dgwm;

namespace {

size_t up256(size_t x) { return (x + 255) & ~size_t(255); }

size_t solve_bytes(const dg_mesh* m) { return dgwm::solve_bytes_mesh(*m); }

}  // namespace

namespace dgwm {
// 9 FP64 and 9 FP32 vectors of the fine level, scalars and partial sums,
// then per coarser multigrid level 4 work vectors and the FP64 and FP32
// inverse diagonals (8 bytes per entry each, so either precision fits).
size_t solve_bytes_mesh(const dg_mesh& m) {
  const size_t n = (size_t)m.n_p;
  size_t b = 9 * up256(n * sizeof(double)) + 9 * up256(n * sizeof(float)) + up256(64 * sizeof(double)) +
             up256(2 * kRedBlocks * sizeof(double));
  for (int l = 1; l < m.mg_nlev; ++l) b += 6 * up256((size_t)m.mg[l].n * sizeof(double));
  return b;
}
}  // namespace dgwm

namespace {

// Work vectors of a solve on mesh m inside a workspace of solve_bytes(m)
// bytes (the layout counted by solve_bytes_mesh).
void carve_solver(Solver& S, const dg_mesh* m, void* ws, hipStream_t stream) {
  S.m = m;
  S.s = stream;
  S.n = m->n_p;
  S.grid = (unsigned)std::min<int64_t>((S.n + 255) / 256, 2048);
  char* w = static_cast<char*>(ws);
  auto take64 = [&](double*& p) { p = reinterpret_cast<double*>(w); w += up256(S.n * sizeof(double)); };
  auto take32 = [&](float*& p) { p = reinterpret_cast<float*>(w); w += up256(S.n * sizeof(float)); };
  take64(S.bp); take64(S.r); take64(S.z); take64(S.zold); take64(S.p); take64(S.q); take64(S.d64); take64(S.t64);
  take64(S.dinv);
  take32(S.r32); take32(S.z32); take32(S.d32); take32(S.t32); take32(S.x32); take32(S.rr32); take32(S.pp32);
  take32(S.qq32); take32(S.dinv32);
  S.sc = reinterpret_cast<double*>(w);
  w += up256(64 * sizeof(double));
  S.part = reinterpret_cast<double*>(w);
  w += up256(2 * kRedBlocks * sizeof(double));
  S.nlev = m->mg_nlev;
  for (int l = 1; l < m->mg_nlev; ++l) {
    const size_t bytes = up256((size_t)m->mg[l].n * sizeof(double));
    Solver::Lv& v = S.lv[l];
    v.n = m->mg[l].n;
    v.x = w; w += bytes;
    v.b = w; w += bytes;
    v.r = w; w += bytes;
    v.t = w; w += bytes;
    v.dinv64 = reinterpret_cast<double*>(w); w += bytes;
    v.dinv32 = reinterpret_cast<float*>(w); w += bytes;
  }
}

// The solve on a workspace that holds at least solve_bytes(m) bytes; every
// byte of it is written before it is read, so its previous contents do not
// matter.  Allocates nothing (the pinned norm slot and its event belong to
// the mesh handle).
int solve_poisson_ws(const dg_mesh* m, const dg_solve_params* sp, const double* b, double* x, void* ws,
                     size_t ws_bytes, dg_solve_stats* st, void* stream) {
  const auto t_start = std::chrono::steady_clock::now();
  if (!m || !sp || !b || !x || !ws) return set_error(DG_ERR_ARG, "mesh/params/b/x/workspace is NULL");
  if (ws_bytes < solve_bytes(m)) return set_error(DG_ERR_WORKSPACE, "solve workspace too small");
  if (!(sp->rtol > 0) || sp->cheb_degree < 1 || sp->coarse_degree < 0 || sp->max_inner < 0 || sp->max_outer < 1)
    return set_error(DG_ERR_ARG, "invalid solve parameters");
  if (b == x) return set_error(DG_ERR_ARG, "b and x must not alias");
  if (m->curved) return set_error(DG_ERR_UNSUPPORTED, "the Poisson operator is built for flat (box) meshes only");
  Solver S;
  carve_solver(S, m, ws, static_cast<hipStream_t>(stream));
  const bool use_mg = sp->multigrid && m->mg_nlev > 1;
  S.nlev = use_mg ? m->mg_nlev : 0;
  double* sc = S.sc;
  enum { RZ0 = 0, RZ1 = 1, PQ = 2, RR = 3, RZX = 4, SUM = 5, NB = 6, SCL = 7, IRZ0 = 8, IRZ1 = 9, IPQ = 10, IRR = 11 };
  int rc;
#define DG_TRY(expr) \
  if ((rc = (expr))) return rc
  hipLaunchKernelGGL((k_recip<double>), dim3(S.grid), dim3(256), 0, S.s, S.dinv, m->diag, S.n);
  hipLaunchKernelGGL((k_recip<float>), dim3(S.grid), dim3(256), 0, S.s, S.dinv32, m->diag, S.n);

  // Chebyshev interval: Lanczos estimate of lmax(D^{-1} A), cached per mesh
  // (and per multigrid level)
  dg_mesh* mm = const_cast<dg_mesh*>(m);
  if (!(mm->lam_max > 0)) {
    DG_TRY(S.lanczos(0, &mm->lam_max));
    S.applies64 = 0;
  }
  if (use_mg) {
    mm->mg[0].lam = mm->lam_max;
    for (int l = 1; l < S.nlev; ++l) {
      const unsigned g = Solver::grid_of(S.lv[l].n);
      hipLaunchKernelGGL((k_recip<double>), dim3(g), dim3(256), 0, S.s, S.lv[l].dinv64, m->mg[l].diag, S.lv[l].n);
      hipLaunchKernelGGL((k_recip<float>), dim3(g), dim3(256), 0, S.s, S.lv[l].dinv32, m->mg[l].diag, S.lv[l].n);
      const bool need = l < S.nlev - 1 || !m->coarse_inv;
      if (need && !(mm->mg[l].lam > 0)) DG_TRY(S.lanczos(l, &mm->mg[l].lam));
    }
  }
  const double lmax = 1.1 * mm->lam_max, lmin = mm->lam_max / 30.0;
  const int deg = sp->cheb_degree;
  const int degc = sp->coarse_degree > 0 ? sp->coarse_degree : deg;

  // b' = b - mean(b), ||b'||
  hipLaunchKernelGGL((k_sum<double>), dim3(S.red(S.n)), dim3(kRedThreads), 0, S.s, b, S.n, S.part);
  DG_TRY(S.red_final(sc + SUM));
  hipLaunchKernelGGL(k_copy_sub_mean, dim3(S.grid), dim3(256), 0, S.s, S.bp, b, S.n, sc + SUM);
  DG_TRY(S.dot(S.bp, S.bp, sc + NB));
  const double nb2 = S.host(sc + NB);
  if (!std::isfinite(nb2)) return set_error(DG_ERR_NONFINITE, "non-finite right-hand side");
  const double nb = std::sqrt(nb2);
  dg_solve_stats stats{};
  if (nb == 0.0) {
    hipLaunchKernelGGL((k_fill<double>), dim3(S.grid), dim3(256), 0, S.s, x, S.n, 0.0);
    DG_TRY(check_hip(hipStreamSynchronize(S.s), "sync"));
    if (st) *st = stats;
    return DG_OK;
  }
  DG_TRY(S.project(x, sc + SUM));

  auto true_residual = [&]() -> double {
    if (S.A64(x, S.q)) return NAN;
    hipLaunchKernelGGL(k_resid, dim3(S.grid), dim3(256), 0, S.s, S.r, S.bp, S.q, S.n);
    if (S.dot(S.r, S.r, sc + RR)) return NAN;
    return std::sqrt(S.host(sc + RR));
  };
  // preconditioner z = M^{-1} r; r32_ready: the FP32 copy of r (and its
  // scale in sc[SCL]) was already written by the residual update
  auto precond = [&](double* zz, bool r32_ready) -> int {
    if (use_mg && !sp->mixed) return S.vcycle<double>(0, zz, S.r, S.q, S.t64, deg, degc);
    if (!use_mg && !sp->mixed) return S.cheb<double>(zz, S.r, S.d64, S.t64, S.dinv, deg, lmin, lmax);
    // normalised FP32 copy of r (||r||^2 is in sc[RR])
    if (!r32_ready)
      hipLaunchKernelGGL(k_to_f32, dim3(S.grid), dim3(256), 0, S.s, S.r32, S.r, S.n, sc + RR, sc + SCL);
    if (use_mg) return S.vcycle<float>(0, S.x32, S.r32, S.rr32, S.t32, deg, degc);
    if (sp->max_inner == 0) {
      int e = S.cheb<float>(S.x32, S.r32, S.d32, S.t32, S.dinv32, deg, lmin, lmax);
      if (e) return e;
    } else {
      // inner FP32 PCG, fixed iteration count (no host synchronisation)
      hipLaunchKernelGGL((k_fill<float>), dim3(S.grid), dim3(256), 0, S.s, S.x32, S.n, 0.0f);
      hipLaunchKernelGGL((k_copy<float>), dim3(S.grid), dim3(256), 0, S.s, S.rr32, S.r32, S.n);
      int e = S.cheb<float>(S.z32, S.rr32, S.d32, S.t32, S.dinv32, deg, lmin, lmax);
      if (e) return e;
      hipLaunchKernelGGL((k_copy<float>), dim3(S.grid), dim3(256), 0, S.s, S.pp32, S.z32, S.n);
      if ((e = S.dot(S.rr32, S.z32, sc + IRZ0))) return e;
      int cur = IRZ0;
      for (int j = 0; j < sp->max_inner; ++j) {
        if ((e = S.A32(S.pp32, S.qq32))) return e;
        if ((e = S.dot(S.pp32, S.qq32, sc + IPQ))) return e;
        hipLaunchKernelGGL((k_update_xr<float>), dim3(S.red(S.n)), dim3(kRedThreads), 0, S.s, S.x32, S.rr32, S.pp32,
                           S.qq32, S.n, sc + cur, sc + IPQ, S.part, (float*)nullptr, (const double*)nullptr,
                           (double*)nullptr);
        ++S.inner_total;
        if (j + 1 == sp->max_inner) break;
        if ((e = S.cheb<float>(S.z32, S.rr32, S.d32, S.t32, S.dinv32, deg, lmin, lmax))) return e;
        const int nxt = cur == IRZ0 ? IRZ1 : IRZ0;
        if ((e = S.dot(S.rr32, S.z32, sc + nxt))) return e;
        hipLaunchKernelGGL((k_update_p<float>), dim3(S.grid), dim3(256), 0, S.s, S.pp32, S.z32, S.n, sc + nxt,
                           (const double*)nullptr, sc + cur);
        cur = nxt;
      }
    }
    return check_hip(hipGetLastError(), "preconditioner");
  };
  // z = M^{-1} r, then r.z -> *rz and (zold != nullptr) r.zold -> *rzx; the
  // FP32 preconditioners return through the scaling pass, which forms the dot
  // products on the way
  auto precond_dots = [&](double* zz, bool r32_ready, const double* zold, double* rz, double* rzx) -> int {
    int e = precond(zz, r32_ready);
    if (e) return e;
    if (!sp->mixed) return zold ? S.dot2(S.r, zz, zold, rz, rzx) : S.dot(S.r, zz, rz);
    hipLaunchKernelGGL(k_from_f32_dot2, dim3(S.red(S.n)), dim3(kRedThreads), 0, S.s, zz, S.x32, sc + SCL, S.r, zold,
                       S.n, S.part);
    return S.red_final(rz, zold ? rzx : nullptr);
  };

  // the residual norm travels to the host through pinned memory, so the
  // next preconditioner can be queued behind the copy and runs while the
  // host waits for the norm (it touches neither x, r nor p)
  double* hsc = m->host_sc;
  hipEvent_t ev = hsc ? m->host_ev : nullptr;

  double rn = true_residual();
  if (!std::isfinite(rn)) return set_error(DG_ERR_NONFINITE, "non-finite residual");
  int it = 0;
  bool converged = rn <= sp->rtol * nb;
  const int max_it = sp->max_outer;
  const int replace_every = 50;
  const bool fused32 = sp->mixed;  // the residual update writes the FP32 copy
  if (!converged) {
    DG_TRY(precond_dots(S.z, false, nullptr, sc + RZ0, nullptr));
    hipLaunchKernelGGL((k_copy<double>), dim3(S.grid), dim3(256), 0, S.s, S.p, S.z, S.n);
    int cur = RZ0;
    for (it = 1; it <= max_it; ++it) {
      DG_TRY(S.A64(S.p, S.q));
      DG_TRY(S.dot(S.p, S.q, sc + PQ));
      hipLaunchKernelGGL((k_update_xr<double>), dim3(S.red(S.n)), dim3(kRedThreads), 0, S.s, x, S.r, S.p, S.q, S.n,
                         sc + cur, sc + PQ, S.part, fused32 ? S.r32 : (float*)nullptr, (const double*)(sc + RR),
                         sc + SCL);
      DG_TRY(S.red_final(sc + RR));
      std::swap(S.z, S.zold);
      const int nxt = cur == RZ0 ? RZ1 : RZ0;
      double rr;
      if (ev) {
        DG_TRY(check_hip(hipMemcpyAsync(hsc, sc + RR, sizeof(double), hipMemcpyDeviceToHost, S.s), "norm copy"));
        DG_TRY(check_hip(hipEventRecord(ev, S.s), "event"));
        DG_TRY(precond_dots(S.z, fused32, S.zold, sc + nxt, sc + RZX));
        DG_TRY(check_hip(hipEventSynchronize(ev), "norm wait"));
        rr = *hsc;
      } else {
        rr = S.host(sc + RR);
        if (std::isfinite(rr)) DG_TRY(precond_dots(S.z, fused32, S.zold, sc + nxt, sc + RZX));
      }
      rn = std::sqrt(rr);
      if (!std::isfinite(rn)) return set_error(DG_ERR_NONFINITE, "non-finite residual");
      if (rn <= sp->rtol * nb || it % replace_every == 0) {
        rn = true_residual();
        if (!std::isfinite(rn)) return set_error(DG_ERR_NONFINITE, "non-finite residual");
        if (rn <= sp->rtol * nb) {
          converged = true;
          break;
        }
        // again from the recomputed residual
        DG_TRY(precond_dots(S.z, false, S.zold, sc + nxt, sc + RZX));
      }
      // flexible (Polak-Ribiere) beta = (r.z - r.z_old) / rz_old
      hipLaunchKernelGGL((k_update_p<double>), dim3(S.grid), dim3(256), 0, S.s, S.p, S.z, S.n, sc + nxt, sc + RZX,
                         sc + cur);
      cur = nxt;
    }
  }
  DG_TRY(S.project(x, sc + SUM));
  DG_TRY(check_hip(hipStreamSynchronize(S.s), "solve synchronize"));
  stats.outer_its = it;
  stats.inner_its_total = S.inner_total;
  stats.op_applies_f64 = S.applies64;
  stats.op_applies_f32 = S.applies32;
  stats.rel_resid = rn / nb;
  stats.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
  if (st) *st = stats;
#undef DG_TRY
  if (!converged) return set_error(DG_ERR_NOT_CONVERGED, "iteration cap reached");
  return DG_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// Batched solves (the serving path): the solves of many meshes advance in
// lockstep, one outer iteration at a time, and every step of an iteration
// (operator applications, smoothing, transfers, vector updates, reductions)
// is one launch over the meshes of the batch (per degree group, up to a
// few per launch, batch.h), with the meshes' descriptors in the kernel
// arguments.  Each mesh runs the same arithmetic as in a batch of one: its
// results do not depend on the others.
// ---------------------------------------------------------------------------
namespace {

// One mesh's part of a batched vector operation.
struct VSeg {
  int64_t blk0;
  int64_t n;     // entries (V_FINAL: partials to add; V_GATHER: output row)
  int64_t nblk;  // workgroups of this segment
  const void* a;
  const void* b;
  const void* c;
  void* d;
  void* e;
  double* sc;    // the mesh's device scalars
  double* part;  // the mesh's reduction partials
  double coef;
};

enum VOp {
  V_SUM, V_SUB_MEAN, V_COPY_SUB_MEAN, V_DOT, V_DOT2, V_FINAL, V_GATHER, V_UPDATE_XR, V_UPDATE_P, V_RESID, V_TO_F32,
  V_FROM_F32_DOT2, V_FILL, V_COPY, V_RECIP64, V_RECIP32, V_HASH, V_JACOBI, V_CHEB_FIRST64, V_CHEB_FIRST32
};

constexpr bool vop_reduces(int op) {
  return op == V_SUM || op == V_DOT || op == V_DOT2 || op == V_UPDATE_XR || op == V_FROM_F32_DOT2;
}

// Workgroups per mesh: reductions use a block count that depends on the
// vector length only (deterministic partials), one block for the finals;
// small vectors get about one entry per thread (latency-bound sizes).
int64_t vop_blocks(int op, int64_t n) {
  if (op == V_FINAL || op == V_GATHER) return 1;
  if (vop_reduces(op)) return red_blocks(n);
  return std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 2048));
}

// i0..i3: scalar slots of the operation (see the cases).
constexpr int kVSegs = 16;  // segments per launch of a vector operation

template <int OP>
__global__ __launch_bounds__(kRedThreads) void k_vop(const SegArr<VSeg, kVSegs> segs, int i0, int i1, int i2, int i3,
                                                     double* __restrict__ gather) {
  __shared__ double sh[kRedThreads / 64];
  const int si = find_seg(segs, (int64_t)blockIdx.x);
  const VSeg S = segs.s[si];
  const int64_t lb = (int64_t)blockIdx.x - S.blk0;
  const int64_t n = S.n, st = S.nblk * (int64_t)blockDim.x;
  const int64_t i00 = lb * (int64_t)blockDim.x + threadIdx.x;
  double* sc = S.sc;
  if constexpr (OP == V_SUM) {  // part = sum a
    const double* a = static_cast<const double*>(S.a);
    double v = 0;
    for (int64_t i = i00; i < n; i += st) v += a[i];
    v = block_reduce(v, sh);
    if (threadIdx.x == 0) S.part[lb] = v;
  } else if constexpr (OP == V_SUB_MEAN) {  // d -= sc[i0] / n
    double* d = static_cast<double*>(S.d);
    const double mean = sc[i0] / (double)n;
    for (int64_t i = i00; i < n; i += st) d[i] -= mean;
  } else if constexpr (OP == V_COPY_SUB_MEAN) {  // d = a - sc[i0] / n
    double* d = static_cast<double*>(S.d);
    const double* a = static_cast<const double*>(S.a);
    const double mean = sc[i0] / (double)n;
    for (int64_t i = i00; i < n; i += st) d[i] = a[i] - mean;
  } else if constexpr (OP == V_DOT) {  // part = a.b
    const double* a = static_cast<const double*>(S.a);
    const double* b = static_cast<const double*>(S.b);
    double v = 0;
    for (int64_t i = i00; i < n; i += st) v += a[i] * b[i];
    v = block_reduce(v, sh);
    if (threadIdx.x == 0) S.part[lb] = v;
  } else if constexpr (OP == V_DOT2) {  // part = a.b, part + nblk = a.c
    const double* a = static_cast<const double*>(S.a);
    const double* b = static_cast<const double*>(S.b);
    const double* c = static_cast<const double*>(S.c);
    double v1 = 0, v2 = 0;
    for (int64_t i = i00; i < n; i += st) {
      v1 += a[i] * b[i];
      v2 += a[i] * c[i];
    }
    v1 = block_reduce(v1, sh);
    __syncthreads();
    v2 = block_reduce(v2, sh);
    if (threadIdx.x == 0) {
      S.part[lb] = v1;
      S.part[S.nblk + lb] = v2;
    }
  } else if constexpr (OP == V_FINAL) {  // sc[i0] = sum of n partials (sc[i1]: the next n, if i1 >= 0)
    double v = 0;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) v += S.part[i];
    v = block_reduce(v, sh);
    if (threadIdx.x == 0) sc[i0] = v;
    if (i1 >= 0) {
      __syncthreads();
      v = 0;
      for (int64_t i = threadIdx.x; i < n; i += blockDim.x) v += S.part[n + i];
      v = block_reduce(v, sh);
      if (threadIdx.x == 0) sc[i1] = v;
    }
  } else if constexpr (OP == V_GATHER) {  // gather[n i2 + j] = sc[i0 + j], j < i1
    for (int j = threadIdx.x; j < i1; j += blockDim.x) gather[n * i2 + j] = sc[i0 + j];
  } else if constexpr (OP == V_UPDATE_XR) {
    // x (d) += alpha p (a), r (e) -= alpha q (b), alpha = sc[i0] / sc[i1]; with c != nullptr the new
    // residual also goes to c in FP32 divided by sqrt(sc[i2]), that divisor stored in sc[i3]; part = r.r
    double* x = static_cast<double*>(S.d);
    double* r = static_cast<double*>(S.e);
    const double* p = static_cast<const double*>(S.a);
    const double* q = static_cast<const double*>(S.b);
    float* r32 = static_cast<float*>(const_cast<void*>(S.c));
    const double alpha = sc[i0] / sc[i1];
    const double nrm = r32 ? sqrt(sc[i2]) : 1.0, inv = 1.0 / nrm;
    double v = 0;
    for (int64_t i = i00; i < n; i += st) {
      x[i] += alpha * p[i];
      const double ri = r[i] - alpha * q[i];
      r[i] = ri;
      if (r32) r32[i] = (float)(ri * inv);
      v += ri * ri;
    }
    v = block_reduce(v, sh);
    if (threadIdx.x == 0) S.part[lb] = v;
    if (r32 && lb == 0 && threadIdx.x == 0) sc[i3] = nrm;
  } else if constexpr (OP == V_UPDATE_P) {  // p (d) = z (a) + beta p, beta = (sc[i0] - sc[i1]) / sc[i2]
    double* p = static_cast<double*>(S.d);
    const double* z = static_cast<const double*>(S.a);
    const double beta = (sc[i0] - (i1 >= 0 ? sc[i1] : 0.0)) / sc[i2];
    for (int64_t i = i00; i < n; i += st) p[i] = z[i] + beta * p[i];
  } else if constexpr (OP == V_RESID) {  // d = a - b
    double* d = static_cast<double*>(S.d);
    const double* a = static_cast<const double*>(S.a);
    const double* b = static_cast<const double*>(S.b);
    for (int64_t i = i00; i < n; i += st) d[i] = a[i] - b[i];
  } else if constexpr (OP == V_TO_F32) {  // d = a / sqrt(sc[i0]) in FP32, the divisor stored in sc[i1]
    float* d = static_cast<float*>(S.d);
    const double* a = static_cast<const double*>(S.a);
    const double nrm = sqrt(sc[i0]), inv = 1.0 / nrm;
    for (int64_t i = i00; i < n; i += st) d[i] = (float)(a[i] * inv);
    if (lb == 0 && threadIdx.x == 0) sc[i1] = nrm;
  } else if constexpr (OP == V_FROM_F32_DOT2) {
    // z (d) = sc[i0] x32 (a); part = r (b) . z, part + nblk = r . zold (c, if not null)
    double* z = static_cast<double*>(S.d);
    const float* x = static_cast<const float*>(S.a);
    const double* r = static_cast<const double*>(S.b);
    const double* zo = static_cast<const double*>(S.c);
    const double s = sc[i0];
    double v1 = 0, v2 = 0;
    for (int64_t i = i00; i < n; i += st) {
      const double zi = s * (double)x[i], ri = r[i];
      z[i] = zi;
      v1 += ri * zi;
      if (zo) v2 += ri * zo[i];
    }
    v1 = block_reduce(v1, sh);
    __syncthreads();
    v2 = block_reduce(v2, sh);
    if (threadIdx.x == 0) {
      S.part[lb] = v1;
      S.part[S.nblk + lb] = v2;
    }
  } else if constexpr (OP == V_FILL) {
    double* d = static_cast<double*>(S.d);
    for (int64_t i = i00; i < n; i += st) d[i] = 0.0;
  } else if constexpr (OP == V_COPY) {
    double* d = static_cast<double*>(S.d);
    const double* a = static_cast<const double*>(S.a);
    for (int64_t i = i00; i < n; i += st) d[i] = a[i];
  } else if constexpr (OP == V_RECIP64) {
    double* d = static_cast<double*>(S.d);
    const double* a = static_cast<const double*>(S.a);
    for (int64_t i = i00; i < n; i += st) d[i] = 1.0 / a[i];
  } else if constexpr (OP == V_RECIP32) {
    float* d = static_cast<float*>(S.d);
    const double* a = static_cast<const double*>(S.a);
    for (int64_t i = i00; i < n; i += st) d[i] = (float)(1.0 / a[i]);
  } else if constexpr (OP == V_HASH) {  // the start vector of the single-mesh Lanczos
    double* d = static_cast<double*>(S.d);
    for (int64_t i = i00; i < n; i += st) {
      uint64_t z = (uint64_t)i + 0x9E3779B97F4A7C15ull;
      z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
      z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
      z ^= z >> 31;
      d[i] = (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
    }
  } else if constexpr (OP == V_JACOBI) {  // d = e = dinv (b) r (a)
    double* d = static_cast<double*>(S.d);
    double* e = static_cast<double*>(S.e);
    const double* r = static_cast<const double*>(S.a);
    const double* di = static_cast<const double*>(S.b);
    for (int64_t i = i00; i < n; i += st) {
      const double v = di[i] * r[i];
      d[i] = v;
      e[i] = v;
    }
  } else if constexpr (OP == V_CHEB_FIRST64 || OP == V_CHEB_FIRST32) {  // d = e = coef dinv (b) r (a)
    using T = typename std::conditional<OP == V_CHEB_FIRST64, double, float>::type;
    T* d = static_cast<T*>(S.d);
    T* e = static_cast<T*>(S.e);
    const T* r = static_cast<const T*>(S.a);
    const T* di = static_cast<const T*>(S.b);
    const T c = (T)S.coef;
    for (int64_t i = i00; i < n; i += st) {
      const T v = c * di[i] * r[i];
      d[i] = v;
      e[i] = v;
    }
  }
}

// Scalar slots of a mesh's sc[] (as in the single solve; 16 and 20..59: Lanczos)
enum { B_RZ0 = 0, B_RZ1 = 1, B_PQ = 2, B_RR = 3, B_RZX = 4, B_SUM = 5, B_NB = 6, B_SCL = 7, B_LSUM = 16, B_LRZ = 20,
       B_LPQ = 40 };
constexpr int kLanczosSteps = 20;
constexpr int kGatherRow = 2 * kLanczosSteps;  // doubles per mesh in the gather array

struct BInst {
  const dg_mesh* m = nullptr;
  Solver S;
  const double* b = nullptr;
  double* x = nullptr;
  int idx = 0;             // position in the caller's arrays (row of the gather array)
  double nb = 0, rn = 0;
  int it = 0;
  int code = DG_OK;
  bool done = false;
  int applies64 = 0, applies32 = 0;
  double seconds = 0;
};

// The launches of one phase of an outer iteration, with their descriptors.
struct Prog {
  std::vector<std::function<int(hipStream_t)>> steps;
  std::vector<BInst*> who;   // meshes whose applies are counted
  std::vector<int> a64, a32;  // level-0 operator applications per run, per entry of who
  void count(BInst* in, bool f64) {
    for (size_t k = 0; k < who.size(); ++k)
      if (who[k] == in) {
        (f64 ? a64 : a32)[k]++;
        return;
      }
    who.push_back(in);
    a64.push_back(f64 ? 1 : 0);
    a32.push_back(f64 ? 0 : 1);
  }
};

using Set = std::vector<BInst*>;

// Pinned host rows for the scalar read-backs, per host thread, kept for the
// thread's lifetime and grown on demand.
struct Pinned {
  char* p = nullptr;
  size_t cap = 0;
  hipEvent_t ev = nullptr;
};
thread_local Pinned tl_pinned;

int pinned_get(size_t bytes, char** out, hipEvent_t* ev) {
  Pinned& P = tl_pinned;
  if (!P.ev && hipEventCreateWithFlags(&P.ev, hipEventDisableTiming) != hipSuccess)
    return set_error(DG_ERR_HIP, "event creation failed");
  if (P.cap < bytes) {
    // grow geometrically: reallocating pinned memory is slow and may wait for the device
    const size_t want = std::max({bytes, 2 * P.cap, size_t(1) << 20});
    if (P.p) (void)hipHostFree(P.p);
    P.p = nullptr;
    P.cap = 0;
    void* q = nullptr;
    if (int rc = check_hip(hipHostMalloc(&q, want, hipHostMallocDefault), "pinned read-back rows")) return rc;
    P.p = static_cast<char*>(q);
    P.cap = want;
  }
  *out = P.p;
  *ev = P.ev;
  return DG_OK;
}

class Batch {
 public:
  std::vector<BInst> I;
  const dg_solve_params* sp = nullptr;
  hipStream_t s = nullptr;
  double* gather = nullptr;   // device: kGatherRow doubles per mesh
  double* rb = nullptr;       // pinned host copy of the gather rows
  hipEvent_t ev = nullptr;
  bool mixed = false;
  int deg0 = 1, degc = 1;

  int run(Prog& P) {
    for (auto& f : P.steps)
      if (int rc = f(s)) return rc;
    for (size_t k = 0; k < P.who.size(); ++k) {
      P.who[k]->applies64 += P.a64[k];
      P.who[k]->applies32 += P.a32[k];
    }
    return DG_OK;
  }
  // copy `rows` gather rows of the set's meshes to the host (asynchronous; wait())
  int readback() {
    if (int rc = check_hip(hipMemcpyAsync(rb, gather, sizeof(double) * kGatherRow * I.size(), hipMemcpyDeviceToHost,
                                          s), "scalar read-back"))
      return rc;
    return check_hip(hipEventRecord(ev, s), "read-back event");
  }
  int wait() { return check_hip(hipEventSynchronize(ev), "read-back wait"); }

  // ---- builders ----
  template <int OP>
  void vop(Prog& P, const Set& set, const std::function<void(VSeg&, BInst&)>& fill, int i0 = -1, int i1 = -1,
           int i2 = -1, int i3 = -1) {
    std::vector<VSeg> v;
    for (BInst* in : set) {
      VSeg g{};
      g.sc = in->S.sc;
      g.part = in->S.part;
      fill(g, *in);
      g.nblk = vop_blocks(OP, g.n);
      v.push_back(g);
    }
    if (v.empty()) return;
    double* ga = gather;
    P.steps.push_back([v, i0, i1, i2, i3, ga](hipStream_t st) -> int {
      for (size_t c0 = 0; c0 < v.size(); c0 += kVSegs) {
        SegArr<VSeg, kVSegs> a{};
        a.n = (int)std::min<size_t>(kVSegs, v.size() - c0);
        int64_t blk = 0;
        for (int i = 0; i < a.n; ++i) {
          a.s[i] = v[c0 + i];
          a.s[i].blk0 = blk;
          blk += a.s[i].nblk;
        }
        hipLaunchKernelGGL((k_vop<OP>), dim3((unsigned)blk), dim3(kRedThreads), 0, st, a, i0, i1, i2, i3, ga);
        if (int rc = check_hip(hipGetLastError(), "batched vector launch")) return rc;
      }
      return DG_OK;
    });
  }
  // sc[o1] (and sc[o2]) = the reduction just built into the partials (n
  // entries each); i0: the scalar slot the reduction's own pass reads
  template <int OP>
  void reduce(Prog& P, const Set& set, const std::function<void(VSeg&, BInst&)>& fill, int o1, int o2 = -1,
              int i0 = -1) {
    vop<OP>(P, set, fill, i0);
    vop<V_FINAL>(P, set, [&](VSeg& g, BInst& in) {
      VSeg t{};
      fill(t, in);
      g.n = vop_blocks(OP, t.n);
    }, o1, o2);
  }
  void gather_rows(Prog& P, const Set& set, int slot, int count) {
    vop<V_GATHER>(P, set, [](VSeg& g, BInst& in) { g.n = in.idx; }, slot, count, kGatherRow);
  }

  template <typename T>
  void poi(Prog& P, int kind, const Set& set, int l, const std::function<void(PoiSeg<T>&, BInst&)>& fill) {
    // one launch per degree group
    std::vector<int> nps;
    for (BInst* in : set)
      if (std::find(nps.begin(), nps.end(), in->m->np_p) == nps.end()) nps.push_back(in->m->np_p);
    for (int np : nps) {
      std::vector<PoiSeg<T>> v;
      for (BInst* in : set) {
        if (in->m->np_p != np) continue;
        PoiSeg<T> g{};
        g.M = poisson_meshdev(in->m, l);
        g.ncell = l > 0 ? in->m->mg[l].ncell : in->m->ncell;
        fill(g, *in);
        g.E.kind = kind;
        v.push_back(g);
        if (l == 0) P.count(in, sizeof(T) == 8);
      }
      P.steps.push_back([v, np, kind](hipStream_t st) {
        return launch_poisson_batched<T>(np, kind, v.data(), (int)v.size(), st);
      });
    }
  }
  template <typename T>
  void xfer(Prog& P, bool restrict_, const Set& set, int l, const std::function<void(TrSeg<T>&, BInst&)>& fill) {
    std::vector<std::pair<int, bool>> groups;
    for (BInst* in : set) {
      const std::pair<int, bool> g(in->m->np_p, mg_full_transfer(in->m, l));
      if (std::find(groups.begin(), groups.end(), g) == groups.end()) groups.push_back(g);
    }
    for (const auto& gr : groups) {
      std::vector<TrSeg<T>> v;
      for (BInst* in : set) {
        if (in->m->np_p != gr.first || mg_full_transfer(in->m, l) != gr.second) continue;
        TrSeg<T> g{};
        g.tr = mg_transfer_geometry(in->m, l);
        g.ncc = in->m->mg[l + 1].ncell;
        fill(g, *in);
        v.push_back(g);
      }
      const int np = gr.first;
      const bool full = gr.second;
      P.steps.push_back([v, np, full, restrict_](hipStream_t st) {
        return restrict_ ? launch_mg_restrict_batched<T>(np, full, v.data(), (int)v.size(), st)
                         : launch_mg_prolong_batched<T>(np, full, v.data(), (int)v.size(), st);
      });
    }
  }
  template <typename T>
  void dense(Prog& P, const Set& set, int l, const std::function<void(DenseSeg<T>&, BInst&)>& fill) {
    std::vector<DenseSeg<T>> v;
    for (BInst* in : set) {
      DenseSeg<T> g{};
      g.n = in->m->mg[l].n;
      g.B = reinterpret_cast<const T*>(sizeof(T) == 8 ? (const void*)in->m->coarse_inv
                                                      : (const void*)in->m->coarse_inv32);
      fill(g, *in);
      v.push_back(g);
    }
    if (v.empty()) return;
    P.steps.push_back([v](hipStream_t st) { return launch_dense_batched<T>(v.data(), (int)v.size(), st); });
  }

  // ---- multigrid V-cycle in lockstep ----
  // level buffers of mesh `in` at level l (l = 0: the caller's four)
  enum Buf { BX = 0, BB = 1, BR = 2, BT = 3 };
  template <typename T>
  struct L0 {
    std::function<T*(BInst&)> b[4];
  };
  template <typename T>
  static T* lvbuf(BInst& in, int l, int which) {
    Solver::Lv& v = in.S.lv[l];
    char* p = which == BX ? v.x : (which == BB ? v.b : (which == BR ? v.r : v.t));
    return reinterpret_cast<T*>(p);
  }
  template <typename T>
  static const T* dinv_l(BInst& in, int l) {
    if (sizeof(T) == 8) return reinterpret_cast<const T*>(l == 0 ? in.S.dinv : in.S.lv[l].dinv64);
    return reinterpret_cast<const T*>(l == 0 ? in.S.dinv32 : in.S.lv[l].dinv32);
  }
  static int64_t n_l(const BInst& in, int l) { return l == 0 ? in.m->n_p : in.m->mg[l].n; }

  // z = Cheb_deg(D^-1 A_l) D^-1 b from a zero start, per mesh interval [lam/lo, hi lam] (Solver::cheb_l)
  template <typename T>
  void cheb_l(Prog& P, const Set& set, int l, const std::function<T*(BInst&, int)>& buf, int deg, double lo_div,
              double hi_mul) {
    // per mesh coefficients
    struct Co { double theta, delta, sigma; };
    auto co = [&](BInst& in) {
      const double lam = in.m->mg[l].lam, lmin = lam / lo_div, lmax = hi_mul * lam;
      Co c;
      c.theta = 0.5 * (lmax + lmin);
      c.delta = 0.5 * (lmax - lmin);
      c.sigma = c.theta / c.delta;
      return c;
    };
    const bool cur_t = ((deg - 1) % 2) != 0;  // the first iterate lands in t for an even step count
    if (deg == 1) {
      vop<sizeof(T) == 8 ? V_CHEB_FIRST64 : V_CHEB_FIRST32>(P, set, [&](VSeg& g, BInst& in) {
        g.n = n_l(in, l);
        g.d = buf(in, cur_t ? BT : BX);
        g.e = buf(in, cur_t ? BX : BT);
        g.a = buf(in, BB);
        g.b = dinv_l<T>(in, l);
        g.coef = 1.0 / co(in).theta;
      });
      return;
    }
    bool cur_is_t = cur_t;
    for (int k = 1; k < deg; ++k) {
      const int cur = cur_is_t ? BT : BX, oth = cur_is_t ? BX : BT;
      const int kk = k;
      poi<T>(P, k == 1 ? kChebFirst : kCheb, set, l, [&](PoiSeg<T>& g, BInst& in) {
        const Co c = co(in);
        double rho = 1.0 / c.sigma, rho_new = 0;
        for (int j = 1; j <= kk; ++j) {
          rho_new = 1.0 / (2.0 * c.sigma - rho);
          if (j < kk) rho = rho_new;
        }
        g.E.b = buf(in, BB);
        g.E.dinv = dinv_l<T>(in, l);
        g.E.c1 = (T)(rho_new * rho);
        g.E.c2 = (T)(2.0 * rho_new / c.delta);
        if (kk == 1) {
          g.p = buf(in, BB);
          g.E.z1 = buf(in, cur);
          g.E.zout = buf(in, oth);
          g.E.c0 = (T)(1.0 / c.theta);
        } else {
          g.p = buf(in, cur);
          g.E.zout = buf(in, oth);
        }
      });
      cur_is_t = !cur_is_t;
    }
  }
  // the same polynomial continued from the current iterate (Solver::cheb_from)
  template <typename T>
  void cheb_from(Prog& P, const Set& set, int l, const std::function<T*(BInst&, int)>& buf, int deg) {
    bool cur_is_t = (deg % 2) != 0;
    for (int k = 0; k < deg; ++k) {
      const int cur = cur_is_t ? BT : BX, oth = cur_is_t ? BX : BT;
      const int kk = k;
      poi<T>(P, kCheb, set, l, [&](PoiSeg<T>& g, BInst& in) {
        const double lam = in.m->mg[l].lam, lmin = lam / kSmoothRange, lmax = 1.1 * lam;
        const double theta = 0.5 * (lmax + lmin), delta = 0.5 * (lmax - lmin), sigma = theta / delta;
        double c1 = 0, c2 = 1.0 / theta, rho = 1.0 / sigma;
        for (int j = 1; j <= kk; ++j) {
          const double rho_new = 1.0 / (2.0 * sigma - rho);
          c1 = rho_new * rho;
          c2 = 2.0 * rho_new / delta;
          rho = rho_new;
        }
        g.p = buf(in, cur);
        g.E.b = buf(in, BB);
        g.E.dinv = dinv_l<T>(in, l);
        g.E.zout = buf(in, oth);
        g.E.c1 = (T)c1;
        g.E.c2 = (T)c2;
      });
      cur_is_t = !cur_is_t;
    }
  }
  template <typename T>
  void vcycle(Prog& P, const Set& set, int l, const std::function<T*(BInst&, int)>& buf) {
    if (set.empty()) return;
    const int deg = l == 0 ? deg0 : degc;
    Set coarse_d, coarse_c, mid;
    for (BInst* in : set) {
      if (l == in->S.nlev - 1) (in->m->coarse_inv ? coarse_d : coarse_c).push_back(in);
      else mid.push_back(in);
    }
    dense<T>(P, coarse_d, l, [&](DenseSeg<T>& g, BInst& in) {
      g.b = buf(in, BB);
      g.x = buf(in, BX);
    });
    if (!coarse_c.empty()) cheb_l<T>(P, coarse_c, l, buf, 4 * deg0, 200.0, 1.1);
    if (mid.empty()) return;
    cheb_l<T>(P, mid, l, buf, deg, kSmoothRange, 1.1);
    poi<T>(P, kResid, mid, l, [&](PoiSeg<T>& g, BInst& in) {
      g.p = buf(in, BX);
      g.y = buf(in, BR);
      g.E.b = buf(in, BB);
    });
    xfer<T>(P, true, mid, l, [&](TrSeg<T>& g, BInst& in) {
      g.in = buf(in, BR);
      g.out = lvbuf<T>(in, l + 1, BB);
    });
    const int lc = l + 1;
    vcycle<T>(P, mid, lc, [lc](BInst& in, int w) { return lvbuf<T>(in, lc, w); });
    xfer<T>(P, false, mid, l, [&](TrSeg<T>& g, BInst& in) {
      g.in = lvbuf<T>(in, lc, BX);
      g.add = buf(in, BX);
      g.out = buf(in, (deg % 2) ? BT : BX);
    });
    cheb_from<T>(P, mid, l, buf, deg);
  }

  // z = M^{-1} r, then r.z -> sc[rz] and (zold) r.zold -> sc[rzx] (precond_dots of the single solve)
  void precond_dots(Prog& P, const Set& set, int zsel, bool r32_ready, int zoldsel, int rz, int rzx) {
    auto zb = [zsel](BInst& in) { return zsel == 0 ? in.S.z : in.S.zold; };
    auto zo = [zoldsel](BInst& in) -> double* { return zoldsel < 0 ? nullptr : (zoldsel == 0 ? in.S.z : in.S.zold); };
    if (mixed) {
      if (!r32_ready)
        vop<V_TO_F32>(P, set, [](VSeg& g, BInst& in) {
          g.n = in.m->n_p;
          g.d = in.S.r32;
          g.a = in.S.r;
        }, B_RR, B_SCL);
      vcycle<float>(P, set, 0, [](BInst& in, int w) {
        return w == BX ? in.S.x32 : (w == BB ? in.S.r32 : (w == BR ? in.S.rr32 : in.S.t32));
      });
      reduce<V_FROM_F32_DOT2>(P, set, [&](VSeg& g, BInst& in) {
        g.n = in.m->n_p;
        g.d = zb(in);
        g.a = in.S.x32;
        g.b = in.S.r;
        g.c = zo(in);
      }, rz, zoldsel >= 0 ? rzx : -1, B_SCL);
      return;
    }
    vcycle<double>(P, set, 0, [zb](BInst& in, int w) {
      return w == BX ? zb(in) : (w == BB ? in.S.r : (w == BR ? in.S.q : in.S.t64));
    });
    if (zoldsel >= 0)
      reduce<V_DOT2>(P, set, [&](VSeg& g, BInst& in) {
        g.n = in.m->n_p;
        g.a = in.S.r;
        g.b = zb(in);
        g.c = zo(in);
      }, rz, rzx);
    else
      reduce<V_DOT>(P, set, [&](VSeg& g, BInst& in) {
        g.n = in.m->n_p;
        g.a = in.S.r;
        g.b = zb(in);
      }, rz);
  }
  // r = b' - A x, r.r -> sc[RR], gathered
  void true_residual(Prog& P, const Set& set) {
    poi<double>(P, kPlain, set, 0, [](PoiSeg<double>& g, BInst& in) {
      g.p = in.x;
      g.y = in.S.q;
    });
    vop<V_RESID>(P, set, [](VSeg& g, BInst& in) {
      g.n = in.m->n_p;
      g.d = in.S.r;
      g.a = in.S.bp;
      g.b = in.S.q;
    });
    reduce<V_DOT>(P, set, [](VSeg& g, BInst& in) {
      g.n = in.m->n_p;
      g.a = in.S.r;
      g.b = in.S.r;
    }, B_RR);
    gather_rows(P, set, B_RR, 1);
  }
  void project_x(Prog& P, const Set& set) {
    reduce<V_SUM>(P, set, [](VSeg& g, BInst& in) {
      g.n = in.m->n_p;
      g.a = in.x;
    }, B_SUM);
    vop<V_SUB_MEAN>(P, set, [](VSeg& g, BInst& in) {
      g.n = in.m->n_p;
      g.d = in.x;
    }, B_SUM);
  }
  // 20 Jacobi-PCG steps on level l of every mesh of the set (Solver::lanczos)
  void lanczos(Prog& P, const Set& set, int l) {
    vop<V_HASH>(P, set, [l](VSeg& g, BInst& in) {
      g.n = n_l(in, l);
      g.d = in.S.r;
    });
    reduce<V_SUM>(P, set, [l](VSeg& g, BInst& in) {
      g.n = n_l(in, l);
      g.a = in.S.r;
    }, B_LSUM);
    vop<V_SUB_MEAN>(P, set, [l](VSeg& g, BInst& in) {
      g.n = n_l(in, l);
      g.d = in.S.r;
    }, B_LSUM);
    vop<V_FILL>(P, set, [l](VSeg& g, BInst& in) {
      g.n = n_l(in, l);
      g.d = in.S.t64;
    });
    for (int k = 0; k < kLanczosSteps; ++k) {
      vop<V_JACOBI>(P, set, [l](VSeg& g, BInst& in) {
        g.n = n_l(in, l);
        g.d = in.S.z;
        g.e = in.S.d64;
        g.a = in.S.r;
        g.b = dinv_l<double>(in, l);
      });
      reduce<V_DOT>(P, set, [l](VSeg& g, BInst& in) {
        g.n = n_l(in, l);
        g.a = in.S.r;
        g.b = in.S.z;
      }, B_LRZ + k);
      if (k == 0)
        vop<V_COPY>(P, set, [l](VSeg& g, BInst& in) {
          g.n = n_l(in, l);
          g.d = in.S.p;
          g.a = in.S.z;
        });
      else
        vop<V_UPDATE_P>(P, set, [l](VSeg& g, BInst& in) {
          g.n = n_l(in, l);
          g.d = in.S.p;
          g.a = in.S.z;
        }, B_LRZ + k, -1, B_LRZ + k - 1);
      poi<double>(P, kPlain, set, l, [](PoiSeg<double>& g, BInst& in) {
        g.p = in.S.p;
        g.y = in.S.q;
      });
      reduce<V_DOT>(P, set, [l](VSeg& g, BInst& in) {
        g.n = n_l(in, l);
        g.a = in.S.p;
        g.b = in.S.q;
      }, B_LPQ + k);
      vop<V_UPDATE_XR>(P, set, [l](VSeg& g, BInst& in) {
        g.n = n_l(in, l);
        g.d = in.S.t64;
        g.e = in.S.r;
        g.a = in.S.p;
        g.b = in.S.q;
      }, B_LRZ + k, B_LPQ + k);
    }
    gather_rows(P, set, B_LRZ, 2 * kLanczosSteps);
  }
};

// lmax from the Lanczos coefficients of one mesh level (as Solver::lanczos)
int lanczos_lmax(const double* h, double* out) {
  constexpr int K = kLanczosSteps;
  double al[K], be[K], diag[K], off[K];
  int kk = 0;
  for (int k = 0; k < K; ++k) {
    const double rz = h[k], pq = h[K + k];
    if (!(rz > 0) || !(pq > 0) || !std::isfinite(rz) || !std::isfinite(pq)) break;
    if (k > 0) be[k - 1] = rz / h[k - 1];
    al[k] = rz / pq;
    kk = k + 1;
  }
  if (kk < 1) return set_error(DG_ERR_NONFINITE, "eigenvalue estimate failed");
  for (int j = 0; j < kk; ++j) {
    diag[j] = 1.0 / al[j] + (j > 0 ? be[j - 1] / al[j - 1] : 0.0);
    if (j + 1 < kk) off[j] = std::sqrt(be[j]) / al[j];
  }
  *out = tridiag_max_eig(diag, off, kk);
  return DG_OK;
}

size_t batch_gather_bytes(int n) { return up256(sizeof(double) * kGatherRow * (size_t)n); }

int solve_batched(const dg_mesh* const* meshes, int n, const dg_solve_params* sp, const double* const* b,
                  double* const* x, void* const* ws, const size_t* ws_bytes, dg_solve_stats* stats, int32_t* codes,
                  void* bws, size_t bws_bytes, hipStream_t s) {
  const auto t0 = std::chrono::steady_clock::now();
  auto since = [&]() { return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count(); };
  if (!meshes || !sp || !b || !x || !ws || !ws_bytes || !bws || n < 1 || n > DG_MAX_BATCH)
    return set_error(DG_ERR_ARG, "batched solve: NULL argument or batch size outside [1, DG_MAX_BATCH]");
  if (!(sp->rtol > 0) || sp->cheb_degree < 1 || sp->coarse_degree < 0 || sp->max_outer < 1)
    return set_error(DG_ERR_ARG, "invalid solve parameters");
  if (!sp->multigrid) return set_error(DG_ERR_UNSUPPORTED, "batched solves run the multigrid preconditioner only");
  for (int i = 0; i < n; ++i) {
    const dg_mesh* m = meshes[i];
    if (!m || !b[i] || !x[i] || !ws[i]) return set_error(DG_ERR_ARG, "batched solve: NULL mesh, vector or workspace");
    if (m->curved) return set_error(DG_ERR_UNSUPPORTED, "the Poisson operator is built for flat (box) meshes only");
    if (m->mg_nlev < 2) return set_error(DG_ERR_UNSUPPORTED, "batched solve: a mesh has no coarser multigrid level");
    if (ws_bytes[i] < solve_bytes(m)) return set_error(DG_ERR_WORKSPACE, "solve workspace too small");
    if (b[i] == x[i]) return set_error(DG_ERR_ARG, "b and x must not alias");
  }
  const size_t gb = batch_gather_bytes(n);
  if (bws_bytes < gb) return set_error(DG_ERR_WORKSPACE, "batched solve: workspace too small");
  Batch B;
  B.sp = sp;
  B.s = s;
  B.mixed = sp->mixed != 0;
  B.deg0 = sp->cheb_degree;
  B.degc = sp->coarse_degree > 0 ? sp->coarse_degree : sp->cheb_degree;
  B.gather = static_cast<double*>(bws);
  char* pin = nullptr;
  if (int rc = pinned_get(gb, &pin, &B.ev)) return rc;
  B.rb = reinterpret_cast<double*>(pin);
  B.I.resize(n);
  Set all;
  for (int i = 0; i < n; ++i) {
    BInst& in = B.I[i];
    in.m = meshes[i];
    carve_solver(in.S, in.m, ws[i], s);
    in.b = b[i];
    in.x = x[i];
    in.idx = i;
    all.push_back(&in);
  }
  int rc;
#define DG_TRY(expr) \
  if ((rc = (expr))) return rc

  // inverse diagonals of every level, b' = b - mean(b), ||b'||^2
  Prog p0;
  B.vop<V_RECIP64>(p0, all, [](VSeg& g, BInst& in) { g.n = in.m->n_p; g.d = in.S.dinv; g.a = in.m->diag; });
  B.vop<V_RECIP32>(p0, all, [](VSeg& g, BInst& in) { g.n = in.m->n_p; g.d = in.S.dinv32; g.a = in.m->diag; });
  for (int l = 1; l < kMaxLevels; ++l) {
    Set sl;
    for (BInst* in : all)
      if (l < in->S.nlev) sl.push_back(in);
    B.vop<V_RECIP64>(p0, sl, [l](VSeg& g, BInst& in) {
      g.n = in.m->mg[l].n; g.d = in.S.lv[l].dinv64; g.a = in.m->mg[l].diag; });
    B.vop<V_RECIP32>(p0, sl, [l](VSeg& g, BInst& in) {
      g.n = in.m->mg[l].n; g.d = in.S.lv[l].dinv32; g.a = in.m->mg[l].diag; });
  }
  B.reduce<V_SUM>(p0, all, [](VSeg& g, BInst& in) { g.n = in.m->n_p; g.a = in.b; }, B_SUM);
  B.vop<V_COPY_SUB_MEAN>(p0, all, [](VSeg& g, BInst& in) { g.n = in.m->n_p; g.d = in.S.bp; g.a = in.b; }, B_SUM);
  B.reduce<V_DOT>(p0, all, [](VSeg& g, BInst& in) { g.n = in.m->n_p; g.a = in.S.bp; g.b = in.S.bp; }, B_NB);
  DG_TRY(B.run(p0));

  // Chebyshev intervals: Lanczos estimates of lmax(D^{-1} A_l), cached per mesh
  for (int l = 0; l < kMaxLevels; ++l) {
    Set need;
    for (BInst* in : all) {
      if (l >= in->S.nlev) continue;
      dg_mesh* mm = const_cast<dg_mesh*>(in->m);
      const bool want = l == 0 ? !(mm->lam_max > 0)
                               : ((l < in->S.nlev - 1 || !mm->coarse_inv) && !(mm->mg[l].lam > 0));
      if (want) need.push_back(in);
    }
    if (need.empty()) continue;
    Prog pl;
    B.lanczos(pl, need, l);
    DG_TRY(B.run(pl));
    DG_TRY(B.readback());
    DG_TRY(B.wait());
    for (BInst* in : need) {
      dg_mesh* mm = const_cast<dg_mesh*>(in->m);
      double lam = 0;
      DG_TRY(lanczos_lmax(B.rb + (size_t)kGatherRow * in->idx, &lam));
      if (l == 0) mm->lam_max = lam;
      else mm->mg[l].lam = lam;
    }
  }
  for (BInst* in : all) {
    dg_mesh* mm = const_cast<dg_mesh*>(in->m);
    mm->mg[0].lam = mm->lam_max;
    in->applies64 = in->applies32 = 0;  // (the estimates are not part of the solve's count)
  }
  // ||b'|| of every mesh (read back after the eigenvalue estimates)
  {
    Prog pg;
    B.gather_rows(pg, all, B_NB, 1);
    DG_TRY(B.run(pg));
    DG_TRY(B.readback());
    DG_TRY(B.wait());
  }
  Set act;
  {
    Set zero;
    for (BInst* in : all) {
      in->nb = std::sqrt(B.rb[(size_t)kGatherRow * in->idx]);
      if (!std::isfinite(in->nb)) {
        in->code = set_error(DG_ERR_NONFINITE, "non-finite right-hand side");
        in->done = true;
      } else if (in->nb == 0.0) {
        zero.push_back(in);
        in->done = true;
      } else {
        act.push_back(in);
      }
    }
    Prog pz;
    B.vop<V_FILL>(pz, zero, [](VSeg& g, BInst& in) { g.n = in.m->n_p; g.d = in.x; });
    DG_TRY(B.run(pz));
  }
  // x to zero mean, true residual of the initial guess
  {
    Prog pi;
    B.project_x(pi, act);
    B.true_residual(pi, act);
    DG_TRY(B.run(pi));
    DG_TRY(B.readback());
    DG_TRY(B.wait());
    Set keep;
    for (BInst* in : act) {
      in->rn = std::sqrt(B.rb[(size_t)kGatherRow * in->idx]);
      if (!std::isfinite(in->rn)) {
        in->code = set_error(DG_ERR_NONFINITE, "non-finite residual");
        in->done = true;
      } else if (in->rn <= sp->rtol * in->nb) {
        in->done = true;
        in->seconds = since();
      } else {
        keep.push_back(in);
      }
    }
    act.swap(keep);
    Prog pp;
    B.precond_dots(pp, act, 0, false, -1, B_RZ0, -1);
    B.vop<V_COPY>(pp, act, [](VSeg& g, BInst& in) { g.n = in.m->n_p; g.d = in.S.p; g.a = in.S.z; });
    DG_TRY(B.run(pp));
  }
  // outer iterations in lockstep; programs are rebuilt when the set changes
  const int replace_every = 50;
  Prog pa[2], pb[2], pc[2];
  bool built = false;
  for (int it = 1; it <= sp->max_outer && !act.empty(); ++it) {
    const int par = it & 1;                       // iteration parity: z and zold swap every iteration
    const int cur = par ? B_RZ0 : B_RZ1, nxt = par ? B_RZ1 : B_RZ0;
    const int zs = par ? 1 : 0, zos = par ? 0 : 1;  // 0: the buffer S.z, 1: S.zold
    if (!built) {
      for (int q = 0; q < 2; ++q) {
        const int c = q ? B_RZ0 : B_RZ1, nx = q ? B_RZ1 : B_RZ0, z = q ? 1 : 0, zo = q ? 0 : 1;
        pa[q] = Prog();
        pb[q] = Prog();
        pc[q] = Prog();
        B.poi<double>(pa[q], kPlain, act, 0, [](PoiSeg<double>& g, BInst& in) { g.p = in.S.p; g.y = in.S.q; });
        B.reduce<V_DOT>(pa[q], act, [](VSeg& g, BInst& in) { g.n = in.m->n_p; g.a = in.S.p; g.b = in.S.q; }, B_PQ);
        const bool m32 = B.mixed;
        B.vop<V_UPDATE_XR>(pa[q], act, [m32](VSeg& g, BInst& in) {
          g.n = in.m->n_p; g.d = in.x; g.e = in.S.r; g.a = in.S.p; g.b = in.S.q;
          g.c = m32 ? (const void*)in.S.r32 : nullptr;
        }, c, B_PQ, B_RR, B_SCL);
        B.vop<V_FINAL>(pa[q], act, [](VSeg& g, BInst& in) { g.n = vop_blocks(V_UPDATE_XR, in.m->n_p); }, B_RR);
        B.gather_rows(pa[q], act, B_RR, 1);
        B.precond_dots(pb[q], act, z, m32, zo, nx, B_RZX);
        B.vop<V_UPDATE_P>(pc[q], act, [z](VSeg& g, BInst& in) {
          g.n = in.m->n_p; g.d = in.S.p; g.a = z == 0 ? in.S.z : in.S.zold;
        }, nx, B_RZX, c);
      }
      built = true;
    }
    DG_TRY(B.run(pa[par]));
    DG_TRY(B.readback());
    DG_TRY(B.run(pb[par]));   // queued behind the read-back; runs while the host waits
    DG_TRY(B.wait());
    Set check, failed;
    for (BInst* in : act) {
      in->it = it;
      in->rn = std::sqrt(B.rb[(size_t)kGatherRow * in->idx]);
      if (!std::isfinite(in->rn)) failed.push_back(in);
      else if (in->rn <= sp->rtol * in->nb || it % replace_every == 0) check.push_back(in);
    }
    Set conv;
    if (!check.empty()) {
      Prog pt;
      B.true_residual(pt, check);
      DG_TRY(B.run(pt));
      DG_TRY(B.readback());
      DG_TRY(B.wait());
      Set again;
      for (BInst* in : check) {
        in->rn = std::sqrt(B.rb[(size_t)kGatherRow * in->idx]);
        if (!std::isfinite(in->rn)) failed.push_back(in);
        else if (in->rn <= sp->rtol * in->nb) conv.push_back(in);
        else again.push_back(in);
      }
      Prog pr;
      B.precond_dots(pr, again, zs, false, zos, nxt, B_RZX);
      DG_TRY(B.run(pr));
    }
    (void)cur;
    DG_TRY(B.run(pc[par]));   // (harmless for the meshes that just converged)
    for (BInst* in : failed) {
      in->code = set_error(DG_ERR_NONFINITE, "non-finite residual");
      in->done = true;
    }
    for (BInst* in : conv) {
      in->done = true;
      in->seconds = since();
    }
    if (!failed.empty() || !conv.empty()) {
      Set keep;
      for (BInst* in : act)
        if (!in->done) keep.push_back(in);
      act.swap(keep);
      built = false;
    }
  }
  for (BInst* in : act) {
    in->code = set_error(DG_ERR_NOT_CONVERGED, "iteration cap reached");
    in->seconds = since();
  }
  // zero-mean solutions
  {
    Set fin;
    for (BInst& in : B.I)
      if (in.code == DG_OK || in.code == DG_ERR_NOT_CONVERGED) fin.push_back(&in);
    Prog pe;
    B.project_x(pe, fin);
    DG_TRY(B.run(pe));
  }
  DG_TRY(check_hip(hipStreamSynchronize(s), "batched solve synchronize"));
  for (BInst& in : B.I) {
    if (codes) codes[in.idx] = in.code;
    if (stats) {
      dg_solve_stats& st = stats[in.idx];
      st = dg_solve_stats{};
      st.outer_its = in.it;
      st.op_applies_f64 = in.applies64;
      st.op_applies_f32 = in.applies32;
      st.rel_resid = in.nb > 0 ? in.rn / in.nb : 0.0;
      st.seconds = in.seconds;
    }
  }
#undef DG_TRY
  return DG_OK;
}

}  // namespace

// Solve workspace of dg_solve_poisson_noalloc: one copy per GPU, held until
// the process ends.  In host code `scratch` only names the symbol; its device
// address comes from hipGetSymbolAddress (scratch_address below).
static __device__ __align__(256) unsigned char scratch[DG_NOALLOC_SOLVE_MAX_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices];  // device address of `scratch` per device (nullptr: not resolved yet)

// Address of `scratch` on the current device, resolved once per device with
// that device current.
int scratch_address(void** out) {
  int dev = -1;
  if (int rc = check_hip(hipGetDevice(&dev), "hipGetDevice")) return rc;
  if (dev < 0 || dev >= kMaxDevices) return set_error(DG_ERR_ARG, "device index outside the supported range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    if (int rc = check_hip(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)")) return rc;
    if (!p) return set_error(DG_ERR_HIP, "hipGetSymbolAddress(scratch) returned NULL");
    g_scratch_dev[dev] = p;
  }
  *out = g_scratch_dev[dev];
  return DG_OK;
}

}  // namespace

extern "C" {

int64_t dg_solve_workspace_bytes(const dg_mesh* m, const dg_solve_params* sp) {
  if (!m || !sp) return set_error(DG_ERR_ARG, "mesh/params is NULL");
  return (int64_t)solve_bytes(m);
}

int dg_solve_poisson(const dg_mesh* m, const dg_solve_params* sp, const double* b, double* x, void* ws,
                     size_t ws_bytes, dg_solve_stats* st, void* stream) {
  return solve_poisson_ws(m, sp, b, x, ws, ws_bytes, st, stream);
}

int dg_solve_poisson_noalloc(const dg_mesh* m, const dg_solve_params* sp, const double* b, double* x,
                             dg_solve_stats* st, void* stream) {
  if (!m || !sp || !b || !x) return set_error(DG_ERR_ARG, "mesh/params/b/x is NULL");
  const size_t need = solve_bytes(m);
  if (need > (size_t)DG_NOALLOC_SOLVE_MAX_BYTES)
    return set_error(DG_ERR_WORKSPACE, "the solve needs more workspace than the built-in scratch holds (" +
                                           std::to_string(need) + " > " +
                                           std::to_string((size_t)DG_NOALLOC_SOLVE_MAX_BYTES) +
                                           " bytes): use dg_solve_poisson with a caller workspace");
  int dev = -1;
  if (int rc = check_hip(hipGetDevice(&dev), "hipGetDevice")) return rc;
  if (dev != m->device) return set_error(DG_ERR_ARG, "the mesh lives on another device than the current one");
  void* ws = nullptr;
  if (int rc = scratch_address(&ws)) return rc;
  return solve_poisson_ws(m, sp, b, x, ws, (size_t)DG_NOALLOC_SOLVE_MAX_BYTES, st, stream);
}

int64_t dg_solve_batch_workspace_bytes(const dg_mesh* const* meshes, int32_t n, const dg_solve_params* sp) {
  if (!meshes || !sp || n < 1 || n > DG_MAX_BATCH)
    return set_error(DG_ERR_ARG, "batched solve: NULL argument or batch size outside [1, DG_MAX_BATCH]");
  for (int i = 0; i < n; ++i)
    if (!meshes[i]) return set_error(DG_ERR_ARG, "batched solve: NULL mesh");
  return (int64_t)batch_gather_bytes(n);
}

int dg_solve_poisson_batched(const dg_mesh* const* meshes, int32_t n, const dg_solve_params* sp,
                             const double* const* b, double* const* x, void* const* ws, const size_t* ws_bytes,
                             dg_solve_stats* stats, int32_t* codes, void* batch_ws, size_t batch_ws_bytes,
                             void* stream) {
  return solve_batched(meshes, n, sp, b, x, ws, ws_bytes, stats, codes, batch_ws, batch_ws_bytes,
                       static_cast<hipStream_t>(stream));
}

}  // extern "C"
