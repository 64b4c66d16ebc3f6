// Internal declarations of the dgwm library (host and device).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "dgwm.h"

namespace dgwm {

constexpr int kMaxP = 8;   // nodes per direction (degree <= 7)
constexpr int kMaxQ = 12;  // Gauss points per direction

// Flat layout of the 1-D tables of one (np, nq, nqy) triple, in doubles.
// Rule "q" (x and z, and y in regular cells) and rule "y" (wall-normal rule
// of enriched cells); both tabulate the same nodal basis.
//   S  [nq][np]  N_i(g_q)          Sd [nq][np]  N_i'(g_q)
//   D  [nq][nq]  L_r'(g_q), L_r the Lagrange polynomial through the Gauss points
//   w  [nq]      Gauss weights     g  [nq]      Gauss points (on [0,1])
//   nd0[np] = N_i'(0), nd1[np] = N_i'(1), gl[np] Gauss-Lobatto nodes,
//   then S, Sd, D, w, g of the y rule.  Offsets of everything before the y
//   rule depend on (np, nq) only.
struct TabLayout {
  int S, Sd, D, w, g;        // q rule
  int nd0, nd1, gl;
  int Sy, Sdy, Dy, wy, gy;   // y rule
  int size;
};

__host__ __device__ constexpr TabLayout tab_layout(int np, int nq, int nqy) {
  TabLayout t{};
  int o = 0;
  t.S = o; o += nq * np;
  t.Sd = o; o += nq * np;
  t.D = o; o += nq * nq;
  t.w = o; o += nq;
  t.g = o; o += nq;
  t.nd0 = o; o += np;
  t.nd1 = o; o += np;
  t.gl = o; o += np;
  t.Sy = o; o += nqy * np;
  t.Sdy = o; o += nqy * np;
  t.Dy = o; o += nqy * nqy;
  t.wy = o; o += nqy;
  t.gy = o; o += nqy;
  t.size = o;
  return t;
}

// 1-D operator tables of the Poisson kernel, stored after the pressure
// tab_layout block: reference mass M_ij = sum_q w_q N_i(g_q) N_j(g_q) and
// stiffness K_ij = sum_q w_q N_i'(g_q) N_j'(g_q) with the Gauss rule of the
// operator, N_i'(0), N_i'(1); first in double, then the same entries in float.
struct PoiOps {
  int M, K, nd0, nd1, n;  // offsets inside one precision block; n entries per block
  int f32;                // offset (in doubles) of the float block
  int size;               // doubles in total
};
__host__ __device__ constexpr PoiOps poi_ops(int np) {
  PoiOps o{};
  o.M = 0;
  o.K = np * np;
  o.nd0 = 2 * np * np;
  o.nd1 = 2 * np * np + np;
  o.n = 2 * np * np + 2 * np;
  o.f32 = o.n;
  o.size = o.n + (o.n + 1) / 2;
  return o;
}

// Points of the enrichment tables of one enriched cell: the volume rule
// nq x nqy x nq, then the six faces f = 2d + s in order.  Face (d,s) has
// tangential directions t1 < t2; its points are q1 + Q1 q2 with Q = nqy for
// the wall-normal direction and nq otherwise.
__host__ __device__ constexpr int psi_face_points(int nq, int nqy, int d) {
  return d == 1 ? nq * nq : nq * nqy;
}
__host__ __device__ constexpr int psi_face_offset(int nq, int nqy, int f) {
  int o = nq * nqy * nq;
  for (int g = 0; g < f; ++g) o += psi_face_points(nq, nqy, g / 2);
  return o;
}
__host__ __device__ constexpr int psi_points(int nq, int nqy) { return psi_face_offset(nq, nqy, 6); }

// Host-side 1-D tables (basis.cpp).
void fill_tables(int np, int nq, int nqy, double* out);
void fill_poisson_ops(int np, int nq, double* out);  // poi_ops(np).size doubles
void gauss_rule(int n, double* x, double* w);
void lobatto_nodes(int n, double* x);

}  // namespace dgwm

namespace dgwm {

// One level of the geometric multigrid hierarchy of the pressure operator.
// Level 0 is the mesh itself; level l+1 merges pairs of cells of level l
// along every direction flagged in (cx, cy, cz).  The tanh-graded wall-normal
// vertices of a coarse level are every second vertex of the finer one, so
// the levels are nested and the coarse space is a subspace of the fine one.
constexpr int kMaxLevels = 12;
constexpr int kMaxCoarseDofs = 1024;  // largest coarsest level solved with the dense inverse
constexpr int kCoarseTarget = 128;    // coarsen while a level has more unknowns than this
struct MgLevel {
  int nx = 0, ny = 0, nz = 0;
  int cx = 0, cy = 0, cz = 0;         // coarsened from level l-1 along x, y, z
  int64_t ncell = 0, n = 0;
  double hx = 0, hz = 0;
  double* hy = nullptr;               // ny cell heights, then their ny reciprocals (device)
  double* diag = nullptr;             // Jacobi diagonal (device, FP64 and FP32)
  float* diag32 = nullptr;
  double lam = 0.0;                   // cached Lanczos estimate of lmax(D^{-1} A)
};

// Support points of van Driest's law (the paper's Appendix A, Table
// tab:psi locations) and U at them, computed at set-up.
struct VdTable {
  static constexpr int N = 9;
  double y[N], psi[N];
};
void vandriest_table(double kappa, double A_plus, VdTable& t);

// Levels of a box mesh: coarsen every direction that has an even cell count
// (and keeps ny >= 2 between walls) while the level has more than
// kCoarseTarget unknowns.
int mg_plan(const dg_mesh_params& P, MgLevel* lv);

}  // namespace dgwm

// Host handle.  All device pointers point into the caller's workspace.
struct dg_mesh {
  dg_mesh_params P;
  int device;
  int64_t ncell, nenr, n_vel, n_p, n_tau;
  int np_u, np_p;
  int n_enr_layers;       // 0, 1 or 2
  int nle;                // enrichment functions per component and enriched cell: (l+1)^3 = 1 or 8
  int lower_slot, upper_slot;  // enriched-layer slot of each wall or -1
  int psi_pts;            // points per enriched cell in the psi tables
  double hx, hz;
  double* host_sc = nullptr;  // pinned host slots for scalars the solver reads back (nullptr: none)
  hipEvent_t host_ev = nullptr;  // marks the copy into host_sc (nullptr: the solver reads synchronously)
  // device
  double* eta;            // ny+1 wall-normal vertex coordinates
  double* tab_u;          // velocity tables (np_u, nq_u, nq_wn)
  double* tab_p;          // pressure tables (np_p, nq_p, nq_p)
  double* tau;            // wall shear stress copy, per wall-face Gauss point
  double* tau_nodes;      // nodal wall shear stress copy [wall][nz][nx] (flat walls)
  int tau_nodal = 0;      // 1: psi was computed from tau_nodes, 0: from tau
  double* ws_part;        // wall shear scratch: [wall][ez][ex][corner][c] (flat walls)
  double* psi;            // [enr][psi_pts][4]: psi, dpsi/dx, dpsi/dy, dpsi/dz
  double* psi_prev;       // the same table before the last wall-shear update
  int32_t* act;           // [enr] enrichment on (1) or switched off (0)
  int32_t* act_prev;      // the same flags before the last wall-shear update
  double* minv;           // inverse 1-D mass matrices [2][np_u][np_u]: x/z rule, wall-normal rule
  double* apoly;          // [enr][2 np_u^3 + 2]: polynomial part of the current psi (inverse mass / projection step cache)
  mutable int apoly_ok = 0;  // apoly matches the current psi table
  double* coup;           // [enr][9 np_u^3 + 6]: projection step couplings of the current psi
  mutable int coup_ok = 0;   // coup matches the current psi table
  double* spec;           // projection step, cells without enrichment: [3][np][np] 1-D factors, then per
                          // distinct layer height (L Z)^T, L^{-T} Z, lambda of the whitened div-div form, then the
                          // int32 layer -> slot map (filled on the first projection step)
  mutable int spec_ok = 0;   // spec filled
  double* diag;           // Poisson diagonal (FP64)
  float* diag32;          // Poisson diagonal (FP32 copy)
  double* hy;             // ny cell heights, then their ny reciprocals
  double lam_max = 0.0;   // cached largest eigenvalue estimate of D^{-1} A (solver)
  // curved lower wall (wall_amp != 0)
  int curved = 0;
  int geo_stride = 0;     // points per cell in the geometry table
  double* geo = nullptr;  // [cell][geo_stride][J^{-1} (9), weight]
  double* meas = nullptr; // [cell][volume, six face areas]
  double* tauF = nullptr; // [cell][face] interior-penalty parameters
  double* wdist = nullptr; // [2][nx+1] distances to the wall of the vertex rows iy = 1 and iy = ny-1
  dgwm::VdTable vd{};     // van Driest support table (psi_kind = DG_PSI_VANDRIEST)
  // pressure multigrid hierarchy (flat meshes): level 0 aliases hy/diag above
  int mg_nlev = 0;
  dgwm::MgLevel mg[dgwm::kMaxLevels];
  // symmetric pseudo-inverse of the coarsest operator (zero-mean range), or
  // nullptr when that level is larger than kMaxCoarseDofs
  double* coarse_inv = nullptr;
  float* coarse_inv32 = nullptr;
};

namespace dgwm {

// Error reporting (api.hip)
int set_error(int code, const std::string& msg);
int check_hip(hipError_t e, const char* what);

// Launchers (defined next to their kernels).  Return DG_OK or an error code.
int launch_psi(const dg_mesh* m, hipStream_t s);
int launch_geometry(const dg_mesh* m, hipStream_t s);
int launch_poisson_diag(const dg_mesh* m, hipStream_t s);
int launch_poisson(const dg_mesh* m, dg_prec prec, const void* p, void* y, hipStream_t s);
// nvec vectors stored vstride entries apart are processed by one launch
int launch_poisson_level(const dg_mesh* m, int level, dg_prec prec, const void* p, void* y, hipStream_t s,
                         int nvec = 1, int64_t vstride = 0);
int launch_poisson_diag_level(const dg_mesh* m, int level, hipStream_t s);
// fused solver steps on level l: r = b - A x, and one Chebyshev step
// zout = z + c1 (z - zprev) + c2 dinv (b - A z), where zout holds the previous
// iterate zprev on entry (zout != z)
template <typename T>
int launch_poisson_resid(const dg_mesh* m, int level, const T* x, const T* b, T* r, hipStream_t s);
template <typename T>
int launch_poisson_cheb(const dg_mesh* m, int level, const T* z, T* zout, const T* b, const T* dinv, T c1, T c2,
                        hipStream_t s);
// the same step from z = c0 dinv b (formed inside the kernel, zprev = 0),
// which is also written to z1
template <typename T>
int launch_poisson_cheb_first(const dg_mesh* m, int level, T c0, T* zout, T* z1, const T* b, const T* dinv, T c1,
                              T c2, hipStream_t s);
// multigrid transfers between level l (fine) and l + 1 (coarse)
int launch_mg_restrict(const dg_mesh* m, int l, dg_prec prec, const void* rf, void* rc, hipStream_t s);
// xo = xf + P xc (xo may be xf)
int launch_mg_prolong_add(const dg_mesh* m, int l, dg_prec prec, const void* xc, const void* xf, void* xo,
                          hipStream_t s);
// x = B b with the dense coarsest-level inverse B (n x n)
int launch_dense_apply(int64_t n, dg_prec prec, const void* B, const void* b, void* x, hipStream_t s);
// device workspace of dg_solve_poisson on mesh m
size_t solve_bytes_mesh(const dg_mesh& m);
// device data of the hierarchy (levels' heights and diagonals, coarse inverse)
int mg_setup(dg_mesh* m, const std::vector<double>& eta0, double* coarse_scr, hipStream_t s);
// convective_only: the residual with nu = 0 (its convective part alone)
int launch_velocity(const dg_mesh* m, dg_prec prec, const void* u, void* r, hipStream_t s,
                    bool convective_only = false);
// eddy viscosity nu_t at every point of the psi tables from the enrichment
// coefficients of u, and out = A u for the multiscale viscous operator
int launch_eddy_viscosity(const dg_mesh* m, const double* u, double c_des, double beta, double* nut, hipStream_t s);
int launch_viscous_multiscale(const dg_mesh* m, const double* nut, const double* u, double* out, hipStream_t s);
// div-div penalty: tau_D per cell from u (tau = true, out: ncell doubles) or out = D u with tau_d
int launch_divdiv(const dg_mesh* m, bool tau, const double* u, const double* tau_d, double dt_over_cr, double* out,
                  hipStream_t s);
int launch_divdiv_curved(const dg_mesh* m, bool tau, const double* u, const double* tau_d, double dt_over_cr,
                         double* out, hipStream_t s);
// out = C u (divergence, pressure layout) or P p (gradient, velocity layout), flat meshes
int launch_divgrad(const dg_mesh* m, bool divergence, const double* in, double* out, hipStream_t s);
int launch_divgrad_curved(const dg_mesh* m, bool divergence, const double* in, double* out, hipStream_t s);
int launch_inverse_mass_curved(const dg_mesh* m, const double* r, double* x, hipStream_t s);
int launch_vorticity_rhs_curved(const dg_mesh* m, const double* u, double* b, hipStream_t s);
int launch_pressure_neumann_curved(const dg_mesh* m, int nh, const double* const* us, const double* const* oms,
                                   const double* beta, const double* f, double* rhs, hipStream_t s);
// element-wise projection step: (M + D) x = M u_hat - scale g per cell, preconditioned CG in each cell
// projection step: spectral tables of every layer (direct solves)
int spectral_layers(const dg_mesh& m, std::vector<int>* map, std::vector<double>* heights);
size_t spectral_table_doubles(const dg_mesh& m);
int ensure_spectral_tables(const dg_mesh* m, hipStream_t s);  // host eigendecompositions on first use
void spectral_pointers(const dg_mesh* m, const double** mats, const double** slots, const int32_t** map);
int launch_spectral_step(const dg_mesh* m, const double* tau_d, const double* u_hat, const double* g, double scale,
                         double* x, hipStream_t s);
int launch_projection_step(const dg_mesh* m, const double* tau_d, const double* u_hat, const double* g, double scale,
                           double* x, hipStream_t s);
// x = M^{-1} r with the velocity mass matrix (flat meshes; x may be r)
int launch_inverse_mass(const dg_mesh* m, const double* r, double* x, hipStream_t s);
// vorticity right-hand side b(v) = (v, curl u)_e and the wall term of the
// pressure Neumann data, added into rhs (kern_step.hip)
int launch_vorticity_rhs(const dg_mesh* m, const double* u, double* b, hipStream_t s);
int launch_pressure_neumann(const dg_mesh* m, int nh, const double* const* us, const double* const* oms,
                            const double* beta, const double* f, double* rhs, hipStream_t s);
// Helmholtz step (helmholtz.hip): workspace bytes and the restarted GMRES solve
int64_t helmholtz_workspace_bytes(const dg_mesh* m, int restart);
int solve_helmholtz(const dg_mesh* m, const double* nut, double gamma, const double* b, double* x, double rtol,
                    int max_iter, int restart, void* ws, size_t ws_bytes, dg_gmres_stats* st, hipStream_t s);
int solve_projection_gmres(const dg_mesh* m, const double* tau_d, const double* b, double* x, double rtol,
                           int max_iter, int restart, void* ws, size_t ws_bytes, dg_gmres_stats* st, hipStream_t s);
// u_new = L2 projection of u_old from the space of psi_prev onto that of psi
int launch_project_velocity(const dg_mesh* m, const double* u_old, double* u_new, hipStream_t s);
// nodal wall shear stress [wall][nz][nx] of the FP64 velocity u (flat walls)
int launch_wall_shear_nodes(const dg_mesh* m, const double* u, double* out, hipStream_t s);
int64_t batch_workspace_bytes(int n);

int launch_velocity_batched(const dg_mesh* const* meshes, int n, dg_prec prec, const void* const* u, void* const* r,
                            void* ws, size_t ws_bytes, hipStream_t s);
bool poisson_supported(int np, int nq);
bool velocity_supported(int np, int nq, int nqy);
bool velocity_l1_supported(int np, int nq, int nqy);  // degree-1 enrichment weights
const char* velocity_l1_combos();
const char* velocity_combos();
const char* poisson_combos();

}  // namespace dgwm
