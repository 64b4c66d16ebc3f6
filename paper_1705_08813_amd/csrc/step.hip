// One time step of the dual-splitting scheme (arXiv 1705.08813, Sec. 4.1
// eqs. convstep, poisson, bc_d_pres, visc; Sec. 4.2 eqs. convstepspat,
// poissonspat, projectionspat, helmholtzspat), FP64, flat walls:
//
//   1 convective step   u^ = ( sum_i alpha_i u^{n-i}
//                              - dt M^{-1} sum_i beta_i F^c(u^{n-i}) ) / gamma0 + dt/gamma0 f
//   2 pressure          A p = -(gamma0/dt) C u^ + int_wall q h_N   (h_N of eq. bc_d_pres with
//                        the vorticities omega^{n-i} = L2 projection of curl u^{n-i})
//   3 projection        (M + D) u^^ = M u^ - dt/gamma0 P p          (D with tau_D from u^n)
//   4 Helmholtz         (gamma0/dt) M u^{n+1} + A_nu(nu_t) u^{n+1} = (gamma0/dt) M u^^
//                        (nu_t from the enrichment of u^n)
//
// Every operator is a library kernel; this file only chains them, with the
// two small combination kernels of steps 1 and 2.  The body force f is a
// constant vector: M^{-1} (v, f) is the constant itself on the polynomial
// unknowns (and 0 on the enrichment ones), which is added directly.
#include <chrono>
#include <cmath>

#include "dgwm_internal.h"

namespace dgwm {

namespace {

size_t up256(size_t b) { return (b + 255) & ~size_t(255); }
// relative residual and iteration cap of the degree-1 projection step's GMRES (the degree-0 path solves
// directly): the enriched cells' mass blocks are near-singular for l = 1 (condition numbers near 1e8), which
// spreads the spectrum of M^{-1} D and makes the iteration long
constexpr double kProjRtol = 1e-12;
constexpr int kProjMaxIter = 50000;
unsigned ew_blocks(int64_t n) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 2048)); }

// s = b0 s + b1 t
__global__ void st_combine(double* __restrict__ s, const double* __restrict__ t, int64_t n, double b0, double b1) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    s[i] = b0 * s[i] + (t ? b1 * t[i] : 0.0);
}

// u^ = (a0 u0 + a1 u1 - dt s) / g0, plus dt/g0 f_c on the polynomial unknowns of component c
__global__ void st_convective(double* __restrict__ uh, const double* __restrict__ u0, const double* __restrict__ u1,
                              const double* __restrict__ s, int64_t n, int64_t enr_off, int64_t np3, double a0,
                              double a1, double dt, double g0, double f0, double f1, double f2) {
  const double ig = 1.0 / g0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    double v = a0 * u0[i] - dt * s[i];
    if (u1) v += a1 * u1[i];
    v *= ig;
    if (i < enr_off) {
      const int c = (int)((i / np3) % 3);
      v += dt * ig * (c == 0 ? f0 : (c == 1 ? f1 : f2));
    }
    uh[i] = v;
  }
}

// y = a y
__global__ void st_scale(double* __restrict__ y, int64_t n, double a) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] *= a;
}

struct StepWs {
  double *s, *t, *uh, *g, *uhh, *om0, *om1, *rhs, *tau_d, *nut;
  void* pws;
  size_t pws_bytes;
  void* hws;
  size_t hws_bytes;
  size_t total;
};

StepWs step_layout(const dg_mesh* m, const dg_step_params* sp, char* base) {
  StepWs W{};
  size_t o = 0;
  const size_t V = up256(sizeof(double) * (size_t)m->n_vel);
  double** vecs[7] = {&W.s, &W.t, &W.uh, &W.g, &W.uhh, &W.om0, &W.om1};
  for (double** v : vecs) {
    *v = reinterpret_cast<double*>(base + o);
    o += V;
  }
  W.rhs = reinterpret_cast<double*>(base + o);
  o += up256(sizeof(double) * (size_t)m->n_p);
  W.tau_d = reinterpret_cast<double*>(base + o);
  o += up256(sizeof(double) * (size_t)m->ncell);
  W.nut = reinterpret_cast<double*>(base + o);
  o += up256(sizeof(double) * (size_t)std::max<int64_t>(1, m->nenr * (int64_t)m->psi_pts));
  W.pws = base + o;
  W.pws_bytes = solve_bytes_mesh(*m);
  o += up256(W.pws_bytes);
  W.hws = base + o;
  W.hws_bytes = (size_t)helmholtz_workspace_bytes(m, sp->helmholtz.restart);
  o += up256(W.hws_bytes);
  W.total = o;
  return W;
}

}  // namespace

}  // namespace dgwm

using namespace dgwm;

extern "C" {

int64_t dg_step_workspace_bytes(const dg_mesh* m, const dg_step_params* sp) {
  if (!m || !sp) return set_error(DG_ERR_ARG, "mesh/params is NULL");
  if (sp->helmholtz.restart < 1 || sp->helmholtz.restart > 100)
    return set_error(DG_ERR_ARG, "GMRES restart outside [1, 100]");
  return (int64_t)step_layout(m, sp, nullptr).total;
}

int dg_dual_splitting_step(const dg_mesh* m, const dg_step_params* sp, const double* u_n, const double* u_nm1,
                           double* u_np1, double* p, void* ws, size_t ws_bytes, dg_step_stats* st, void* stream) {
  const auto t0 = std::chrono::steady_clock::now();
  if (!m || !sp || !u_n || !u_np1 || !p || !ws) return set_error(DG_ERR_ARG, "mesh/params/u_n/u_np1/p/ws is NULL");
  if (m->curved) return set_error(DG_ERR_UNSUPPORTED, "the dual-splitting step is built for flat walls only");
  if (m->P.omit_step_tables)
    return set_error(DG_ERR_UNSUPPORTED, "the mesh was set up without projection-step tables (omit_step_tables)");
  if (sp->order != 1 && sp->order != 2) return set_error(DG_ERR_ARG, "order must be 1 or 2");
  if (sp->order == 2 && !u_nm1) return set_error(DG_ERR_ARG, "order 2 needs u_nm1");
  if (!(sp->dt > 0) || !(sp->gamma0 > 0) || !std::isfinite(sp->dt + sp->gamma0) || !(sp->dt_over_cr >= 0))
    return set_error(DG_ERR_ARG, "invalid time-step parameters");
  if (u_np1 == u_n || u_np1 == u_nm1) return set_error(DG_ERR_ARG, "u_np1 must not alias u_n or u_nm1");
  if (sp->helmholtz.restart < 1 || sp->helmholtz.restart > 100)
    return set_error(DG_ERR_ARG, "GMRES restart outside [1, 100]");
  if (st) st->projection_its = 0;
  const StepWs W = step_layout(m, sp, static_cast<char*>(ws));
  if (ws_bytes < W.total) return set_error(DG_ERR_WORKSPACE, "step workspace too small");
  const hipStream_t s = static_cast<hipStream_t>(stream);
  const int J = sp->order;
  const int64_t nv = m->n_vel, npr = m->n_p;
  const int64_t np3 = (int64_t)m->np_u * m->np_u * m->np_u;
  const int64_t enr_off = m->ncell * 3 * np3;
  const double* us[2] = {u_n, J == 2 ? u_nm1 : nullptr};
  int rc;
#define DG_TRY(expr) \
  if ((rc = (expr))) return rc

  // 1 convective step: s = M^{-1} sum_i beta_i F^c(u^{n-i}), then u^
  DG_TRY(launch_velocity(m, DG_F64, u_n, W.s, s, true));
  if (J == 2) DG_TRY(launch_velocity(m, DG_F64, u_nm1, W.t, s, true));
  hipLaunchKernelGGL(st_combine, dim3(ew_blocks(nv)), dim3(256), 0, s, W.s, J == 2 ? W.t : nullptr, nv, sp->beta[0],
                     sp->beta[1]);
  DG_TRY(launch_inverse_mass(m, W.s, W.s, s));
  hipLaunchKernelGGL(st_convective, dim3(ew_blocks(nv)), dim3(256), 0, s, W.uh, u_n, J == 2 ? u_nm1 : nullptr, W.s,
                     nv, enr_off, np3, sp->alpha[0], sp->alpha[1], sp->dt, sp->gamma0, sp->f[0], sp->f[1], sp->f[2]);
  DG_TRY(check_hip(hipGetLastError(), "convective step"));

  // 2 pressure: rhs = -(gamma0/dt) C u^ + wall term of the Neumann data
  DG_TRY(launch_divgrad(m, true, W.uh, W.rhs, s));
  hipLaunchKernelGGL(st_scale, dim3(ew_blocks(npr)), dim3(256), 0, s, W.rhs, npr, -sp->gamma0 / sp->dt);
  DG_TRY(launch_vorticity_rhs(m, u_n, W.om0, s));
  DG_TRY(launch_inverse_mass(m, W.om0, W.om0, s));
  if (J == 2) {
    DG_TRY(launch_vorticity_rhs(m, u_nm1, W.om1, s));
    DG_TRY(launch_inverse_mass(m, W.om1, W.om1, s));
  }
  const double* oms[2] = {W.om0, W.om1};
  DG_TRY(launch_pressure_neumann(m, J, us, oms, sp->beta, sp->f, W.rhs, s));
  dg_solve_stats pst{};
  rc = dg_solve_poisson(m, &sp->poisson, W.rhs, p, W.pws, W.pws_bytes, &pst, stream);
  if (st) st->poisson = pst;
  if (rc) return rc;

  // 3 projection: (M + D) u^^ = M u^ - dt/gamma0 P p, tau_D from u^n
  DG_TRY(launch_divgrad(m, false, p, W.g, s));
  DG_TRY(launch_divdiv(m, true, u_n, nullptr, sp->dt_over_cr, W.tau_d, s));
  if (m->nle == 1 || m->nenr == 0) {
    DG_TRY(launch_projection_step(m, W.tau_d, W.uh, W.g, sp->dt / sp->gamma0, W.uhh, s));
  } else {
    // degree-1 enrichment weights: u^^ + M^{-1} D u^^ = u^ - dt/gamma0 M^{-1} P p by the restarted GMRES of
    // the Helmholtz step (block diagonal, the same workspace), from u^
    DG_TRY(launch_inverse_mass(m, W.g, W.t, s));
    DG_TRY(check_hip(hipMemcpyAsync(W.s, W.uh, sizeof(double) * nv, hipMemcpyDeviceToDevice, s), "projection rhs"));
    hipLaunchKernelGGL(st_combine, dim3(ew_blocks(nv)), dim3(256), 0, s, W.s, W.t, nv, 1.0, -sp->dt / sp->gamma0);
    DG_TRY(check_hip(hipMemcpyAsync(W.uhh, W.uh, sizeof(double) * nv, hipMemcpyDeviceToDevice, s), "initial guess"));
    dg_gmres_stats pst{};
    rc = solve_projection_gmres(m, W.tau_d, W.s, W.uhh, kProjRtol, kProjMaxIter, sp->helmholtz.restart, W.hws,
                                W.hws_bytes, &pst, s);
    if (st) st->projection_its = pst.iterations;
    if (rc) return rc;
  }

  // 4 Helmholtz: nu_t from u^n, initial guess u^^
  if (m->nenr > 0) DG_TRY(launch_eddy_viscosity(m, u_n, sp->c_des, sp->beta_des, W.nut, s));
  DG_TRY(check_hip(hipMemcpyAsync(u_np1, W.uhh, sizeof(double) * nv, hipMemcpyDeviceToDevice, s), "initial guess"));
  dg_gmres_stats hst{};
  rc = solve_helmholtz(m, m->nenr > 0 ? W.nut : nullptr, sp->gamma0 / sp->dt, W.uhh, u_np1, sp->helmholtz.rtol,
                       sp->helmholtz.max_iter, sp->helmholtz.restart, W.hws, W.hws_bytes, &hst, s);
  if (st) {
    st->helmholtz = hst;
    st->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
#undef DG_TRY
  return rc;
}

}  // extern "C"
