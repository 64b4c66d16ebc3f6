// C ABI entry points: argument checking, mesh set-up on the host, workspace
// layout, and dispatch to the kernels.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "dgwm_internal.h"

namespace dgwm {

namespace {
thread_local std::string g_err;

bool aligned256(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 255u) == 0; }

struct WsLayout {
  size_t eta, hy, tab_u, tab_p, tau, tau_nodes, ws_part, psi, psi_prev, act, act_prev, minv, apoly, coup, spec, diag, diag32, geo,
      meas, tauF, wdist;
  size_t mg_hy[kMaxLevels], mg_diag[kMaxLevels], mg_diag32[kMaxLevels];
  size_t cinv, cinv32, cscr;  // coarsest pseudo-inverse (FP64, FP32) and its assembly scratch
  size_t total;
};

size_t up256(size_t x) { return (x + 255) & ~size_t(255); }


// Inverse of the 1-D mass matrix M_ij = sum_q w_q N_i(g_q) N_j(g_q) of a
// Gauss rule with nq >= np points (symmetric positive definite), by
// Gauss-Jordan elimination with partial pivoting; S is [nq][np], out [np][np].
void inverse_mass_1d(int np, int nq, const double* S, const double* w, double* out) {
  std::vector<double> a(np * 2 * np, 0.0);
  for (int i = 0; i < np; ++i) {
    for (int j = 0; j < np; ++j) {
      double m = 0.0;
      for (int q = 0; q < nq; ++q) m += w[q] * S[q * np + i] * S[q * np + j];
      a[i * 2 * np + j] = m;
    }
    a[i * 2 * np + np + i] = 1.0;
  }
  for (int c = 0; c < np; ++c) {
    int piv = c;
    for (int r = c + 1; r < np; ++r)
      if (std::fabs(a[r * 2 * np + c]) > std::fabs(a[piv * 2 * np + c])) piv = r;
    if (piv != c)
      for (int k = 0; k < 2 * np; ++k) std::swap(a[c * 2 * np + k], a[piv * 2 * np + k]);
    const double d = 1.0 / a[c * 2 * np + c];
    for (int k = 0; k < 2 * np; ++k) a[c * 2 * np + k] *= d;
    for (int r = 0; r < np; ++r) {
      if (r == c) continue;
      const double f = a[r * 2 * np + c];
      if (f == 0.0) continue;
      for (int k = 0; k < 2 * np; ++k) a[r * 2 * np + k] -= f * a[c * 2 * np + k];
    }
  }
  for (int i = 0; i < np; ++i)
    for (int j = 0; j < np; ++j) out[i * np + j] = a[i * 2 * np + np + j];
}

// The current psi table and activity flags become the previous ones; the
// next psi launch overwrites the (old) previous buffers.
void keep_previous_space(dg_mesh* m) {
  std::swap(m->psi, m->psi_prev);
  std::swap(m->act, m->act_prev);
  m->apoly_ok = 0;
  m->coup_ok = 0;
}

}  // namespace

int set_error(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

int check_hip(hipError_t e, const char* what) {
  if (e == hipSuccess) return DG_OK;
  return set_error(DG_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

namespace {

// Derived sizes; returns an error code for invalid parameters.
int derive(const dg_mesh_params& P, dg_mesh& m) {
  if (P.nx < 1 || P.ny < 1 || P.nz < 1) return set_error(DG_ERR_ARG, "cell counts must be >= 1");
  if (!P.fully_periodic && P.ny < 2) return set_error(DG_ERR_ARG, "ny must be >= 2 when the channel has walls");
  if (P.k_u < 1 || P.k_u + 1 > kMaxP || P.k_p < 1 || P.k_p + 1 > kMaxP)
    return set_error(DG_ERR_ARG, "polynomial degree out of range");
  if (P.nq_u < 1 || P.nq_u > kMaxQ || P.nq_p < 1 || P.nq_p > kMaxQ || P.nq_wn < 1 || P.nq_wn > kMaxQ)
    return set_error(DG_ERR_ARG, "quadrature size out of range");
  if (!(P.Lx > 0) || !(P.Lz > 0) || !(P.nu > 0) || !(P.kappa > 0) || !(P.gamma >= 0) ||
      !std::isfinite(P.Lx + P.Lz + P.nu + P.kappa + P.B + P.gamma + P.wall_amp))
    return set_error(DG_ERR_ARG, "geometry or material parameter invalid");
  if (!(P.ip_factor_u > 0) || !(P.ip_factor_p > 0) || !(P.wall_ip_mult > 0))
    return set_error(DG_ERR_ARG, "penalty factors must be positive");
  if (P.psi_kind != DG_PSI_SPALDING && P.psi_kind != DG_PSI_VANDRIEST)
    return set_error(DG_ERR_ARG, "psi_kind must be DG_PSI_SPALDING or DG_PSI_VANDRIEST");
  if (P.psi_kind == DG_PSI_VANDRIEST && !(P.A_plus > 0 && std::isfinite(P.A_plus)))
    return set_error(DG_ERR_ARG, "A_plus must be positive and finite");
  if (!(P.yplus_off >= 0) || !std::isfinite(P.yplus_off))
    return set_error(DG_ERR_ARG, "yplus_off must be >= 0 and finite");
  if (P.enrich_degree != 0 && P.enrich_degree != 1) return set_error(DG_ERR_ARG, "enrich_degree must be 0 or 1");
  if (P.omit_step_tables != 0 && P.omit_step_tables != 1) return set_error(DG_ERR_ARG, "omit_step_tables must be 0 or 1");
  if (P.enrich_degree == 1 && P.wall_amp != 0.0)
    return set_error(DG_ERR_UNSUPPORTED, "degree-1 enrichment weights are built for flat walls only");
  if (P.wall_amp != 0.0 && P.fully_periodic) return set_error(DG_ERR_ARG, "a curved wall needs walls");
  if (!(std::fabs(P.wall_amp) < 0.9)) return set_error(DG_ERR_ARG, "wall amplitude must be below 0.9");
  m.P = P;
  m.ncell = (int64_t)P.nx * P.ny * P.nz;
  if (m.ncell > INT32_MAX) return set_error(DG_ERR_ARG, "more than 2^31 - 1 cells");
  m.np_u = P.k_u + 1;
  m.np_p = P.k_p + 1;
  m.lower_slot = m.upper_slot = -1;
  m.n_enr_layers = 0;
  if (!P.fully_periodic) {
    if (P.enrich_lower) m.lower_slot = m.n_enr_layers++;
    if (P.enrich_upper) m.upper_slot = m.n_enr_layers++;
  }
  m.nenr = (int64_t)P.nx * P.nz * m.n_enr_layers;
  m.nle = P.enrich_degree ? 8 : 1;
  m.n_vel = m.ncell * 3 * (int64_t)m.np_u * m.np_u * m.np_u + 3 * (int64_t)m.nle * m.nenr;
  m.n_p = m.ncell * (int64_t)m.np_p * m.np_p * m.np_p;
  m.n_tau = 2 * (int64_t)P.nz * P.nx * P.nq_u * P.nq_u;
  m.psi_pts = psi_points(P.nq_u, P.nq_wn);
  m.hx = P.Lx / P.nx;
  m.hz = P.Lz / P.nz;
  m.curved = P.wall_amp != 0.0;
  m.geo_stride = m.curved ? psi_points(P.nq_u, std::max(P.nq_u, P.nq_wn)) : 0;
  m.mg_nlev = m.curved ? 0 : mg_plan(P, m.mg);
  const int nqw_eff = m.nenr > 0 ? P.nq_wn : -1;
  if (m.nenr > 0 && !velocity_supported(m.np_u, P.nq_u, nqw_eff))
    return set_error(DG_ERR_UNSUPPORTED, std::string("velocity (k_u+1, nq_u, nq_wn) not compiled; have ") +
                                             velocity_combos());
  if (m.nenr > 0 && m.nle != 1 && !velocity_l1_supported(m.np_u, P.nq_u, P.nq_wn))
    return set_error(DG_ERR_UNSUPPORTED, std::string("degree-1 enrichment weights: (k_u+1, nq_u, nq_wn) not "
                                                     "compiled; have ") + velocity_l1_combos());
  if (m.nenr == 0) {
    bool any = false;
    for (int w = 1; w <= kMaxQ && !any; ++w) any = velocity_supported(m.np_u, P.nq_u, w);
    if (!any)
      return set_error(DG_ERR_UNSUPPORTED, std::string("velocity (k_u+1, nq_u) not compiled; have ") +
                                               velocity_combos());
  }
  if (!poisson_supported(m.np_p, P.nq_p))
    return set_error(DG_ERR_UNSUPPORTED, std::string("pressure (k_p+1, nq_p) not compiled; have ") +
                                             poisson_combos());
  return DG_OK;
}

WsLayout layout(const dg_mesh& m) {
  WsLayout L{};
  size_t o = 0;
  L.eta = o; o = up256(o + sizeof(double) * (m.P.ny + 1));
  L.hy = o; o = up256(o + sizeof(double) * 2 * m.P.ny);  // heights, then their reciprocals
  L.tab_u = o;
  o = up256(o + sizeof(double) * (tab_layout(m.np_u, m.P.nq_u, m.P.nq_wn).size + m.P.nq_u + m.P.nq_wn));
  L.tab_p = o;
  o = up256(o + sizeof(double) * (tab_layout(m.np_p, m.P.nq_p, m.P.nq_p).size + poi_ops(m.np_p).size));
  L.tau = o; o = up256(o + sizeof(double) * m.n_tau);
  const size_t nwall = m.curved || m.P.fully_periodic ? 0 : 2 * (size_t)m.P.nz * m.P.nx;
  L.tau_nodes = o; o = up256(o + sizeof(double) * nwall);
  L.ws_part = o; o = up256(o + sizeof(double) * 12 * nwall);
  L.psi = o; o = up256(o + sizeof(double) * 4 * (size_t)m.nenr * m.psi_pts);
  L.psi_prev = o; o = up256(o + sizeof(double) * 4 * (size_t)m.nenr * m.psi_pts);
  L.act = o; o = up256(o + sizeof(int32_t) * (size_t)m.nenr);
  L.act_prev = o; o = up256(o + sizeof(int32_t) * (size_t)m.nenr);
  L.minv = o; o = up256(o + sizeof(double) * 2 * m.np_u * m.np_u);
  {
    const size_t np3 = (size_t)m.np_u * m.np_u * m.np_u;  // l = 1: 8 coefficient vectors and the 8 x 8 inverse Gram matrix
    L.apoly = o; o = up256(o + sizeof(double) * (size_t)m.nenr * (m.nle == 1 ? 2 * np3 + 2 : 8 * np3 + 64));
  }
  // projection-step tables (left out on request)
  const bool st = !m.P.omit_step_tables;
  L.coup = o; o = up256(o + (st ? sizeof(double) * (size_t)m.nenr * (9 * m.np_u * m.np_u * m.np_u + 6) : 0));
  L.spec = o; o = up256(o + (st ? sizeof(double) * spectral_table_doubles(m) : 0));
  L.diag = o; o = up256(o + sizeof(double) * m.n_p);
  L.diag32 = o; o = up256(o + sizeof(float) * m.n_p);
  L.geo = o; o = up256(o + sizeof(double) * 10 * (size_t)m.ncell * m.geo_stride);
  L.meas = o; o = up256(o + sizeof(double) * (m.curved ? 7 * (size_t)m.ncell : 0));
  L.tauF = o; o = up256(o + sizeof(double) * (m.curved ? 6 * (size_t)m.ncell : 0));
  L.wdist = o; o = up256(o + sizeof(double) * (m.curved ? 2 * (size_t)(m.P.nx + 1) : 0));
  for (int l = 1; l < m.mg_nlev; ++l) {
    L.mg_hy[l] = o; o = up256(o + sizeof(double) * 2 * m.mg[l].ny);
    L.mg_diag[l] = o; o = up256(o + sizeof(double) * m.mg[l].n);
    L.mg_diag32[l] = o; o = up256(o + sizeof(float) * m.mg[l].n);
  }
  const int64_t nc = m.mg_nlev > 0 ? m.mg[m.mg_nlev - 1].n : 0;
  const bool dense = m.mg_nlev > 0 && nc <= kMaxCoarseDofs;
  L.cinv = o; o = up256(o + (dense ? sizeof(double) * nc * nc : 0));
  L.cinv32 = o; o = up256(o + (dense ? sizeof(float) * nc * nc : 0));
  L.cscr = o; o = up256(o + (dense ? 2 * sizeof(double) * nc * nc : 0));
  L.total = o;
  return L;
}

}  // namespace
}  // namespace dgwm

using namespace dgwm;

extern "C" {

const char* dg_last_error(void) { return g_err.c_str(); }

const char* dg_build_info(void) {
  static std::string s;
  s = std::string("gfx950; ") + velocity_combos() + "; " + poisson_combos();
  return s.c_str();
}

int64_t dg_mesh_workspace_bytes(const dg_mesh_params* params) {
  if (!params) return set_error(DG_ERR_ARG, "params is NULL");
  dg_mesh m{};
  int rc = derive(*params, m);
  if (rc) return rc;
  return (int64_t)layout(m).total;
}

int64_t dg_solve_workspace_bytes_for(const dg_mesh_params* params, const dg_solve_params* sp) {
  if (!params || !sp) return set_error(DG_ERR_ARG, "params/solve params is NULL");
  dg_mesh m{};
  int rc = derive(*params, m);
  if (rc) return rc;
  return (int64_t)solve_bytes_mesh(m);
}

int dg_setup_mesh(const dg_mesh_params* params, const double* tau_w_host, void* workspace, size_t ws_bytes,
                  void* stream, dg_mesh** out) {
  if (!params || !out) return set_error(DG_ERR_ARG, "params/out is NULL");
  *out = nullptr;
  dg_mesh* m = new dg_mesh();
  int rc = derive(*params, *m);
  if (rc) {
    delete m;
    return rc;
  }
  const WsLayout W = layout(*m);
  if (!workspace || ws_bytes < W.total) {
    delete m;
    return set_error(DG_ERR_WORKSPACE, "mesh workspace missing or too small (need " + std::to_string(W.total) +
                                           " bytes)");
  }
  if (!aligned256(workspace)) {
    delete m;
    return set_error(DG_ERR_ARG, "workspace must be 256-byte aligned");
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  if ((rc = check_hip(hipGetDevice(&m->device), "hipGetDevice"))) {
    delete m;
    return rc;
  }
  char* base = static_cast<char*>(workspace);
  m->eta = reinterpret_cast<double*>(base + W.eta);
  m->hy = reinterpret_cast<double*>(base + W.hy);
  m->tab_u = reinterpret_cast<double*>(base + W.tab_u);
  m->tab_p = reinterpret_cast<double*>(base + W.tab_p);
  m->tau = reinterpret_cast<double*>(base + W.tau);
  m->tau_nodes = reinterpret_cast<double*>(base + W.tau_nodes);
  m->ws_part = reinterpret_cast<double*>(base + W.ws_part);
  m->psi = reinterpret_cast<double*>(base + W.psi);
  m->psi_prev = reinterpret_cast<double*>(base + W.psi_prev);
  m->act = reinterpret_cast<int32_t*>(base + W.act);
  m->act_prev = reinterpret_cast<int32_t*>(base + W.act_prev);
  m->minv = reinterpret_cast<double*>(base + W.minv);
  m->apoly = reinterpret_cast<double*>(base + W.apoly);
  m->spec = reinterpret_cast<double*>(base + W.spec);
  m->coup = reinterpret_cast<double*>(base + W.coup);
  m->diag = reinterpret_cast<double*>(base + W.diag);
  m->diag32 = reinterpret_cast<float*>(base + W.diag32);
  for (int l = 0; l < m->mg_nlev; ++l) {
    if (l == 0) continue;
    m->mg[l].hy = reinterpret_cast<double*>(base + W.mg_hy[l]);
    m->mg[l].diag = reinterpret_cast<double*>(base + W.mg_diag[l]);
    m->mg[l].diag32 = reinterpret_cast<float*>(base + W.mg_diag32[l]);
  }
  if (m->mg_nlev > 0 && m->mg[m->mg_nlev - 1].n <= kMaxCoarseDofs) {
    m->coarse_inv = reinterpret_cast<double*>(base + W.cinv);
    m->coarse_inv32 = reinterpret_cast<float*>(base + W.cinv32);
  }
  if (m->curved) {
    m->geo = reinterpret_cast<double*>(base + W.geo);
    m->meas = reinterpret_cast<double*>(base + W.meas);
    m->tauF = reinterpret_cast<double*>(base + W.tauF);
    m->wdist = reinterpret_cast<double*>(base + W.wdist);
  }

  const dg_mesh_params& P = m->P;
  // wall-normal vertices: tanh grading (paper Sec. 5.1)
  std::vector<double> eta(P.ny + 1), hy(2 * P.ny);  // heights, then their reciprocals
  for (int j = 0; j <= P.ny; ++j) {
    const double t = 2.0 * j / P.ny - 1.0;
    eta[j] = P.gamma > 0 ? std::tanh(P.gamma * t) / std::tanh(P.gamma) : t;
  }
  for (int j = 0; j < P.ny; ++j) {
    hy[j] = eta[j + 1] - eta[j];
    hy[P.ny + j] = 1.0 / hy[j];
  }
  const TabLayout Lu = tab_layout(m->np_u, P.nq_u, P.nq_wn);
  std::vector<double> tu(Lu.size + P.nq_u + P.nq_wn), tp(tab_layout(m->np_p, P.nq_p, P.nq_p).size + poi_ops(m->np_p).size);
  fill_tables(m->np_u, P.nq_u, P.nq_wn, tu.data());
  for (int q = 0; q < P.nq_u; ++q) tu[Lu.size + q] = tu[Lu.g + q];
  for (int q = 0; q < P.nq_wn; ++q) tu[Lu.size + P.nq_u + q] = tu[Lu.gy + q];
  fill_tables(m->np_p, P.nq_p, P.nq_p, tp.data());
  fill_poisson_ops(m->np_p, P.nq_p, tp.data() + tab_layout(m->np_p, P.nq_p, P.nq_p).size);
  std::vector<double> tau(m->n_tau, 1.0);
  if (tau_w_host) {
    for (int64_t i = 0; i < m->n_tau; ++i) {
      if (!(tau_w_host[i] > 0.0) || !std::isfinite(tau_w_host[i])) {
        delete m;
        return set_error(DG_ERR_ARG, "tau_w must be positive and finite");
      }
      tau[i] = tau_w_host[i];
    }
  }
  rc = check_hip(hipMemcpyAsync(m->eta, eta.data(), sizeof(double) * eta.size(), hipMemcpyHostToDevice, s), "copy");
  if (!rc) rc = check_hip(hipMemcpyAsync(m->hy, hy.data(), sizeof(double) * hy.size(), hipMemcpyHostToDevice, s), "copy");
  if (!rc) rc = check_hip(hipMemcpyAsync(m->tab_u, tu.data(), sizeof(double) * tu.size(), hipMemcpyHostToDevice, s), "copy");
  if (!rc) rc = check_hip(hipMemcpyAsync(m->tab_p, tp.data(), sizeof(double) * tp.size(), hipMemcpyHostToDevice, s), "copy");
  if (!rc) rc = check_hip(hipMemcpyAsync(m->tau, tau.data(), sizeof(double) * tau.size(), hipMemcpyHostToDevice, s), "copy");
  // curved wall: distances of the wall-adjacent vertex rows to the closest
  // wall vertex (paper Sec. 3.2: y_B is the distance to the closest wall node)
  std::vector<double> wd;
  if (m->curved) {
    const double hx = m->hx, amp = P.wall_amp, Lx = P.Lx;
    auto yw = [&](double x) { return -1.0 + amp * std::cos(2.0 * M_PI * x / Lx); };
    auto ymap = [&](double x, double et) { return yw(x) + 0.5 * (et + 1.0) * (1.0 - yw(x)); };
    wd.assign(2 * (P.nx + 1), 0.0);
    for (int ix = 0; ix <= P.nx; ++ix) {
      const double x = ix * hx, y = ymap(x, eta[1]);
      double best = 1e300;
      for (int jx = 0; jx < P.nx; ++jx)
        for (int img = -1; img <= 1; ++img) {
          const double dx = x - (jx * hx + img * Lx), dy = y - yw(jx * hx);
          best = std::min(best, std::sqrt(dx * dx + dy * dy));
        }
      wd[ix] = best;
      wd[P.nx + 1 + ix] = std::fabs(1.0 - ymap(x, eta[P.ny - 1]));
    }
    if (!rc) rc = check_hip(hipMemcpyAsync(m->wdist, wd.data(), sizeof(double) * wd.size(), hipMemcpyHostToDevice, s), "copy");
    if (!rc) rc = launch_geometry(m, s);
  }
  if (P.psi_kind == DG_PSI_VANDRIEST) vandriest_table(P.kappa, P.A_plus, m->vd);
  // without a switch-off threshold every enriched cell stays on: both flag
  // arrays are set once and the activity kernel never runs
  std::vector<int32_t> ones(m->nenr > 0 && !(P.yplus_off > 0) ? m->nenr : 0, 1);
  if (!rc && !ones.empty())
    rc = check_hip(hipMemcpyAsync(m->act, ones.data(), sizeof(int32_t) * ones.size(), hipMemcpyHostToDevice, s),
                   "copy");
  if (!rc) rc = launch_psi(m, s);
  // the previous-space tables start as copies of the current ones (a
  // projection before any update is the identity)
  if (!rc && m->nenr > 0)
    rc = check_hip(hipMemcpyAsync(m->psi_prev, m->psi, sizeof(double) * 4 * (size_t)m->nenr * m->psi_pts,
                                  hipMemcpyDeviceToDevice, s), "copy");
  if (!rc && m->nenr > 0)
    rc = check_hip(hipMemcpyAsync(m->act_prev, m->act, sizeof(int32_t) * (size_t)m->nenr, hipMemcpyDeviceToDevice,
                                  s), "copy");
  std::vector<double> minv(2 * m->np_u * m->np_u);
  inverse_mass_1d(m->np_u, P.nq_u, tu.data() + Lu.S, tu.data() + Lu.w, minv.data());
  inverse_mass_1d(m->np_u, P.nq_wn, tu.data() + Lu.Sy, tu.data() + Lu.wy, minv.data() + m->np_u * m->np_u);
  if (!rc)
    rc = check_hip(hipMemcpyAsync(m->minv, minv.data(), sizeof(double) * minv.size(), hipMemcpyHostToDevice, s),
                   "copy");
  if (!rc && !m->curved) rc = launch_poisson_diag(m, s);
  if (!rc && m->mg_nlev > 0) {
    m->mg[0].hy = m->hy;
    m->mg[0].diag = m->diag;
    m->mg[0].diag32 = m->diag32;
    rc = mg_setup(m, eta, reinterpret_cast<double*>(base + W.cscr), s);
  }
  if (!rc) rc = check_hip(hipStreamSynchronize(s), "setup synchronize");
  if (rc) {
    delete m;
    return rc;
  }
  // pinned slot for the solver's residual norms (the solver reads them back
  // synchronously when this allocation is refused)
  if (hipHostMalloc(reinterpret_cast<void**>(&m->host_sc), 64 * sizeof(double), hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    m->host_sc = nullptr;
  }
  if (m->host_sc && hipEventCreateWithFlags(&m->host_ev, hipEventDisableTiming) != hipSuccess) {
    (void)hipGetLastError();
    m->host_ev = nullptr;
  }
  *out = m;
  return DG_OK;
}

int dg_update_wall_shear(dg_mesh* m, const double* tau_w_dev, void* stream) {
  if (!m || !tau_w_dev) return set_error(DG_ERR_ARG, "mesh/tau_w is NULL");
  hipStream_t s = static_cast<hipStream_t>(stream);
  int rc = check_hip(hipMemcpyAsync(m->tau, tau_w_dev, sizeof(double) * m->n_tau, hipMemcpyDeviceToDevice, s),
                     "tau copy");
  if (rc) return rc;
  m->tau_nodal = 0;
  keep_previous_space(m);
  return launch_psi(m, s);
}

int dg_wall_shear_nodes(const dg_mesh* m, const double* u, double* tau_nodes, void* stream) {
  if (!m || !u || !tau_nodes) return set_error(DG_ERR_ARG, "mesh/u/tau_nodes is NULL");
  if (m->curved || m->P.fully_periodic)
    return set_error(DG_ERR_UNSUPPORTED, "nodal wall shear stress: flat no-slip walls only");
  if (static_cast<const void*>(u) == static_cast<const void*>(tau_nodes))
    return set_error(DG_ERR_ARG, "u and tau_nodes must not alias");
  if (!aligned256(u) || !aligned256(tau_nodes)) return set_error(DG_ERR_ARG, "u and tau_nodes must be 256-byte aligned");
  return launch_wall_shear_nodes(m, u, tau_nodes, static_cast<hipStream_t>(stream));
}

int dg_update_wall_shear_nodes(dg_mesh* m, const double* tau_nodes, void* stream) {
  if (!m || !tau_nodes) return set_error(DG_ERR_ARG, "mesh/tau_nodes is NULL");
  if (m->curved || m->P.fully_periodic)
    return set_error(DG_ERR_UNSUPPORTED, "nodal wall shear stress: flat no-slip walls only");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const size_t n = 2 * (size_t)m->P.nz * m->P.nx;
  int rc = check_hip(hipMemcpyAsync(m->tau_nodes, tau_nodes, sizeof(double) * n, hipMemcpyDeviceToDevice, s),
                     "tau_nodes copy");
  if (rc) return rc;
  m->tau_nodal = 1;
  keep_previous_space(m);
  return launch_psi(m, s);
}

int dg_project_velocity(const dg_mesh* m, const double* u_old, double* u_new, void* stream) {
  if (!m || !u_old || !u_new) return set_error(DG_ERR_ARG, "mesh/u_old/u_new is NULL");
  if (m->curved) return set_error(DG_ERR_UNSUPPORTED, "projection onto the refreshed space: flat meshes only");
  if (!aligned256(u_old) || !aligned256(u_new)) return set_error(DG_ERR_ARG, "u_old and u_new must be 256-byte aligned");
  return launch_project_velocity(m, u_old, u_new, static_cast<hipStream_t>(stream));
}

int dg_apply_inverse_mass(const dg_mesh* m, const double* r, double* x, void* stream) {
  if (!m || !r || !x) return set_error(DG_ERR_ARG, "mesh/r/x is NULL");
  if (!aligned256(r) || !aligned256(x)) return set_error(DG_ERR_ARG, "r and x must be 256-byte aligned");
  return launch_inverse_mass(m, r, x, static_cast<hipStream_t>(stream));
}

int dg_apply_pressure_gradient(const dg_mesh* m, const double* p, double* g, void* stream) {
  if (!m || !p || !g) return set_error(DG_ERR_ARG, "mesh/p/g is NULL");
  if (static_cast<const void*>(p) == static_cast<const void*>(g)) return set_error(DG_ERR_ARG, "p and g must not alias");
  if (!aligned256(p) || !aligned256(g)) return set_error(DG_ERR_ARG, "p and g must be 256-byte aligned");
  return launch_divgrad(m, false, p, g, static_cast<hipStream_t>(stream));
}

int dg_apply_velocity_divergence(const dg_mesh* m, const double* u, double* c, void* stream) {
  if (!m || !u || !c) return set_error(DG_ERR_ARG, "mesh/u/c is NULL");
  if (static_cast<const void*>(u) == static_cast<const void*>(c)) return set_error(DG_ERR_ARG, "u and c must not alias");
  if (!aligned256(u) || !aligned256(c)) return set_error(DG_ERR_ARG, "u and c must be 256-byte aligned");
  return launch_divgrad(m, true, u, c, static_cast<hipStream_t>(stream));
}

int dg_divdiv_tau(const dg_mesh* m, const double* u, double dt_over_cr, double* tau_d, void* stream) {
  if (!m || !u || !tau_d) return set_error(DG_ERR_ARG, "mesh/u/tau_d is NULL");
  if (!(dt_over_cr >= 0) || !std::isfinite(dt_over_cr)) return set_error(DG_ERR_ARG, "dt/Cr must be >= 0 and finite");
  if (static_cast<const void*>(u) == static_cast<const void*>(tau_d)) return set_error(DG_ERR_ARG, "u and tau_d must not alias");
  if (!aligned256(u) || !aligned256(tau_d)) return set_error(DG_ERR_ARG, "u and tau_d must be 256-byte aligned");
  return launch_divdiv(m, true, u, nullptr, dt_over_cr, tau_d, static_cast<hipStream_t>(stream));
}

int dg_apply_divdiv(const dg_mesh* m, const double* tau_d, const double* u, double* out, void* stream) {
  if (!m || !tau_d || !u || !out) return set_error(DG_ERR_ARG, "mesh/tau_d/u/out is NULL");
  if (u == out) return set_error(DG_ERR_ARG, "u and out must not alias");
  if (!aligned256(u) || !aligned256(out) || !aligned256(tau_d))
    return set_error(DG_ERR_ARG, "tau_d, u and out must be 256-byte aligned");
  return launch_divdiv(m, false, u, tau_d, 0.0, out, static_cast<hipStream_t>(stream));
}

int dg_projection_step(const dg_mesh* m, const double* tau_d, const double* u_hat, const double* g, double scale,
                       double* x, void* stream) {
  if (!m || !tau_d || !u_hat || !g || !x) return set_error(DG_ERR_ARG, "mesh/tau_d/u_hat/g/x is NULL");
  if (m->curved) return set_error(DG_ERR_UNSUPPORTED, "projection step: flat meshes only");
  if (m->nle != 1) return set_error(DG_ERR_UNSUPPORTED, "built for l = 0 enrichment weights only");
  if (!std::isfinite(scale)) return set_error(DG_ERR_ARG, "scale must be finite");
  if (x == u_hat || x == g || x == tau_d) return set_error(DG_ERR_ARG, "x must not alias u_hat, g or tau_d");
  if (!aligned256(tau_d) || !aligned256(u_hat) || !aligned256(g) || !aligned256(x))
    return set_error(DG_ERR_ARG, "tau_d, u_hat, g and x must be 256-byte aligned");
  return launch_projection_step(m, tau_d, u_hat, g, scale, x, static_cast<hipStream_t>(stream));
}

int64_t dg_eddy_viscosity_points(const dg_mesh* m) {
  if (!m) return set_error(DG_ERR_ARG, "mesh is NULL");
  return m->nenr * (int64_t)m->psi_pts;
}

int dg_eddy_viscosity(const dg_mesh* m, const double* u, double c_des, double beta, double* nut, void* stream) {
  if (!m || !u || !nut) return set_error(DG_ERR_ARG, "mesh/u/nut is NULL");
  if (m->curved) return set_error(DG_ERR_UNSUPPORTED, "eddy viscosity: flat meshes only");
  if (!(c_des > 0) || !std::isfinite(c_des) || !(beta > 0) || !std::isfinite(beta))
    return set_error(DG_ERR_ARG, "c_des and beta must be positive and finite");
  if (static_cast<const void*>(u) == static_cast<const void*>(nut)) return set_error(DG_ERR_ARG, "u and nut must not alias");
  if (!aligned256(u) || !aligned256(nut)) return set_error(DG_ERR_ARG, "u and nut must be 256-byte aligned");
  return launch_eddy_viscosity(m, u, c_des, beta, nut, static_cast<hipStream_t>(stream));
}

int dg_apply_viscous_multiscale(const dg_mesh* m, const double* nut, const double* u, double* out, void* stream) {
  if (!m || !u || !out || (!nut && m->nenr > 0)) return set_error(DG_ERR_ARG, "mesh/nut/u/out is NULL");
  if (m->curved) return set_error(DG_ERR_UNSUPPORTED, "multiscale viscous operator: flat meshes only");
  if (u == out || (nut && (nut == u || nut == out))) return set_error(DG_ERR_ARG, "u, out and nut must not alias");
  if (!aligned256(u) || !aligned256(out) || (nut && !aligned256(nut)))
    return set_error(DG_ERR_ARG, "nut, u and out must be 256-byte aligned");
  return launch_viscous_multiscale(m, nut, u, out, static_cast<hipStream_t>(stream));
}

int dg_enrichment_active(const dg_mesh* m, int32_t* flags, void* stream) {
  if (!m || !flags) return set_error(DG_ERR_ARG, "mesh/flags is NULL");
  if (m->nenr == 0) return DG_OK;
  return check_hip(hipMemcpyAsync(flags, m->act, sizeof(int32_t) * (size_t)m->nenr, hipMemcpyDeviceToDevice,
                                  static_cast<hipStream_t>(stream)),
                   "activity copy");
}

int64_t dg_num_dofs(const dg_mesh* m, int field) {
  if (!m) return set_error(DG_ERR_ARG, "mesh is NULL");
  if (field == 0) return m->n_vel;
  if (field == 1) return m->n_p;
  return set_error(DG_ERR_ARG, "field must be 0 (velocity) or 1 (pressure)");
}

int64_t dg_num_enriched(const dg_mesh* m) {
  if (!m) return set_error(DG_ERR_ARG, "mesh is NULL");
  return m->nenr;
}

void dg_destroy_mesh(dg_mesh* m) {
  if (m && m->host_ev) (void)hipEventDestroy(m->host_ev);
  if (m && m->host_sc) (void)hipHostFree(m->host_sc);
  delete m;
}

int dg_apply_velocity_residual(const dg_mesh* m, dg_prec prec, const void* u, void* r, void* stream) {
  if (!m || !u || !r) return set_error(DG_ERR_ARG, "mesh/u/r is NULL");
  if (prec != DG_F64 && prec != DG_F32) return set_error(DG_ERR_ARG, "unknown precision");
  if (u == r) return set_error(DG_ERR_ARG, "u and r must not alias");
  if (!aligned256(u) || !aligned256(r)) return set_error(DG_ERR_ARG, "u and r must be 256-byte aligned");
  return launch_velocity(m, prec, u, r, static_cast<hipStream_t>(stream));
}

int dg_apply_convective(const dg_mesh* m, dg_prec prec, const void* u, void* r, void* stream) {
  if (!m || !u || !r) return set_error(DG_ERR_ARG, "mesh/u/r is NULL");
  if (prec != DG_F64 && prec != DG_F32) return set_error(DG_ERR_ARG, "unknown precision");
  if (u == r) return set_error(DG_ERR_ARG, "u and r must not alias");
  if (!aligned256(u) || !aligned256(r)) return set_error(DG_ERR_ARG, "u and r must be 256-byte aligned");
  return launch_velocity(m, prec, u, r, static_cast<hipStream_t>(stream), true);
}

int64_t dg_batch_workspace_bytes(int32_t n) {
  if (n < 1 || n > DG_MAX_BATCH) return set_error(DG_ERR_ARG, "batch size must be in [1, DG_MAX_BATCH]");
  return batch_workspace_bytes(n);
}

int dg_apply_velocity_residual_batched(const dg_mesh* const* meshes, int32_t n, dg_prec prec, const void* const* u,
                                       void* const* r, void* workspace, size_t ws_bytes, void* stream) {
  if (!meshes || !u || !r || !workspace) return set_error(DG_ERR_ARG, "meshes/u/r/workspace is NULL");
  if (n < 1 || n > DG_MAX_BATCH) return set_error(DG_ERR_ARG, "batch size must be in [1, DG_MAX_BATCH]");
  if (prec != DG_F64 && prec != DG_F32) return set_error(DG_ERR_ARG, "unknown precision");
  if (!aligned256(workspace)) return set_error(DG_ERR_ARG, "workspace must be 256-byte aligned");
  for (int i = 0; i < n; ++i) {
    if (!meshes[i] || !u[i] || !r[i]) return set_error(DG_ERR_ARG, "a batch entry has a NULL mesh/u/r");
    if (u[i] == r[i]) return set_error(DG_ERR_ARG, "u and r of a batch entry must not alias");
    if (!aligned256(u[i]) || !aligned256(r[i])) return set_error(DG_ERR_ARG, "u and r must be 256-byte aligned");
    if (meshes[i]->nle != 1)
      return set_error(DG_ERR_UNSUPPORTED, "the batched residual is built for l = 0 enrichment weights only");
    for (int j = 0; j < i; ++j)
      if (r[j] == r[i]) return set_error(DG_ERR_ARG, "two batch entries share an output vector");
  }
  return launch_velocity_batched(meshes, n, prec, u, r, workspace, ws_bytes, static_cast<hipStream_t>(stream));
}

int dg_apply_poisson(const dg_mesh* m, dg_prec prec, const void* p, void* y, void* stream) {
  if (!m || !p || !y) return set_error(DG_ERR_ARG, "mesh/p/y is NULL");
  if (m->curved) return set_error(DG_ERR_UNSUPPORTED, "the Poisson operator is built for flat (box) meshes only");
  if (prec != DG_F64 && prec != DG_F32) return set_error(DG_ERR_ARG, "unknown precision");
  if (p == y) return set_error(DG_ERR_ARG, "p and y must not alias");
  if (!aligned256(p) || !aligned256(y)) return set_error(DG_ERR_ARG, "p and y must be 256-byte aligned");
  return launch_poisson(m, prec, p, y, static_cast<hipStream_t>(stream));
}

int dg_mg_levels(const dg_mesh* m, int32_t* out, int32_t cap) {
  if (!m) return set_error(DG_ERR_ARG, "mesh is NULL");
  if (cap < 0 || (cap > 0 && !out)) return set_error(DG_ERR_ARG, "out is NULL or cap negative");
  for (int l = 0; l < m->mg_nlev && l < cap; ++l) {
    const MgLevel& v = m->mg[l];
    const int32_t row[6] = {v.nx, v.ny, v.nz, v.cx, v.cy, v.cz};
    for (int i = 0; i < 6; ++i) out[6 * l + i] = row[i];
  }
  return m->mg_nlev;
}

int dg_mg_transfer(const dg_mesh* m, int32_t level, int32_t direction, dg_prec prec, const void* in,
                   const void* add, void* out, void* stream) {
  if (!m || !in || !out || (direction == 1 && !add)) return set_error(DG_ERR_ARG, "mesh/in/add/out is NULL");
  if (m->curved) return set_error(DG_ERR_UNSUPPORTED, "curved meshes have no multigrid hierarchy");
  if (level < 0 || level + 1 >= m->mg_nlev) return set_error(DG_ERR_ARG, "level outside the hierarchy");
  if (prec != DG_F64 && prec != DG_F32) return set_error(DG_ERR_ARG, "unknown precision");
  if (in == out) return set_error(DG_ERR_ARG, "in and out must not alias");
  const hipStream_t s = static_cast<hipStream_t>(stream);
  if (direction == 0) return launch_mg_restrict(m, level, prec, in, out, s);
  if (direction == 1) return launch_mg_prolong_add(m, level, prec, in, add, out, s);
  return set_error(DG_ERR_ARG, "unknown transfer direction");
}

int dg_poisson_diagonal(const dg_mesh* m, double* d, void* stream) {
  if (!m || !d) return set_error(DG_ERR_ARG, "mesh/d is NULL");
  if (m->curved) return set_error(DG_ERR_UNSUPPORTED, "the Poisson operator is built for flat (box) meshes only");
  return check_hip(hipMemcpyAsync(d, m->diag, sizeof(double) * m->n_p, hipMemcpyDeviceToDevice,
                                  static_cast<hipStream_t>(stream)),
                   "diagonal copy");
}

}  // extern "C"
