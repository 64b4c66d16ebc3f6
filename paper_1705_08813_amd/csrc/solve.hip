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
#include <mutex>
#include <string>
#include <cmath>
#include <vector>

#include "dgwm_internal.h"

namespace dgwm {

namespace {

constexpr int kRedBlocks = 2048;  // eight blocks per CU keep enough loads in flight
constexpr double kSmoothRange = 20.0;  // multigrid smoother interval [lmax / 20, 1.1 lmax]
constexpr int kRedThreads = 256;

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

// a.b1 and a.b2 in one pass (partials of the second at part + kRedBlocks)
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
    part[kRedBlocks + blockIdx.x] = v2;
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

// out[j] = sum of the kRedBlocks partials at part + j kRedBlocks, j < nout
// (one block, fixed order).
__global__ __launch_bounds__(kRedThreads) void k_final(const double* __restrict__ part, double* __restrict__ out,
                                                       double* __restrict__ out2) {
  __shared__ double sh[kRedThreads / 64];
  double v = 0;
  for (int i = threadIdx.x; i < kRedBlocks; i += blockDim.x) v += part[i];
  v = block_reduce(v, sh);
  if (threadIdx.x == 0) *out = v;
  if (!out2) return;
  __syncthreads();
  v = 0;
  for (int i = threadIdx.x; i < kRedBlocks; i += blockDim.x) v += part[kRedBlocks + i];
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
// r.zold (second set at part + kRedBlocks)
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
    part[kRedBlocks + blockIdx.x] = v2;
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

  int red_final(double* out, double* out2 = nullptr) {
    hipLaunchKernelGGL(k_final, dim3(1), dim3(kRedThreads), 0, s, part, out, out2);
    return check_hip(hipGetLastError(), "reduce");
  }
  // a.b1 -> out1, a.b2 -> out2 in one pass over a
  int dot2(const double* a, const double* b1, const double* b2, double* out1, double* out2) {
    hipLaunchKernelGGL(k_dot2, dim3(kRedBlocks), dim3(kRedThreads), 0, s, a, b1, b2, n, part);
    return red_final(out1, out2);
  }
  template <typename TA, typename TB>
  int dot(const TA* a, const TB* b, double* out, int64_t nn = -1) {
    hipLaunchKernelGGL((k_dot<TA, TB>), dim3(kRedBlocks), dim3(kRedThreads), 0, s, a, b, nn < 0 ? n : nn, part);
    return red_final(out);
  }
  template <typename T>
  int project(T* a, double* sum, int64_t nn = -1) {
    if (nn < 0) nn = n;
    hipLaunchKernelGGL((k_sum<T>), dim3(kRedBlocks), dim3(kRedThreads), 0, s, a, nn, part);
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
    hipLaunchKernelGGL((k_update_xr<double>), dim3(kRedBlocks), dim3(kRedThreads), 0, s, t64, r, p, q, nn, RZ + k,
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
  S.m = m;
  S.s = static_cast<hipStream_t>(stream);
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
  const bool use_mg = sp->multigrid && m->mg_nlev > 1;
  S.nlev = use_mg ? m->mg_nlev : 0;
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
  hipLaunchKernelGGL((k_sum<double>), dim3(kRedBlocks), dim3(kRedThreads), 0, S.s, b, S.n, S.part);
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
        hipLaunchKernelGGL((k_update_xr<float>), dim3(kRedBlocks), dim3(kRedThreads), 0, S.s, S.x32, S.rr32, S.pp32,
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
    hipLaunchKernelGGL(k_from_f32_dot2, dim3(kRedBlocks), dim3(kRedThreads), 0, S.s, zz, S.x32, sc + SCL, S.r, zold,
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
      hipLaunchKernelGGL((k_update_xr<double>), dim3(kRedBlocks), dim3(kRedThreads), 0, S.s, x, S.r, S.p, S.q, S.n,
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

}  // extern "C"
