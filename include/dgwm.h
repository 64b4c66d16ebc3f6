/*
 * dgwm.h -- C ABI of the MI355X (gfx950) library for the enriched
 * discontinuous-Galerkin operators of the multiscale RANS/LES wall model of
 * Krank, Kronbichler & Wall (arXiv 1705.08813).
 *
 * Conventions shared by every entry point
 * ----------------------------------------
 *  - Return value: 0 on success, a negative DG_ERR_* code otherwise; the
 *    message of the last failure on the calling thread is dg_last_error().
 *    No C++ exception crosses this boundary.
 *  - Device pointers are HIP device (or managed) addresses on the device that
 *    is current when the call is made; they must be 256-byte aligned and
 *    must not alias one another unless stated.  Host pointers are ordinary
 *    CPU memory.  The library never frees caller memory.
 *  - `stream` is a hipStream_t passed as void* (NULL = the legacy default
 *    stream).  Apply calls only enqueue work and return; results are ready
 *    when the stream has drained.  Inputs are never modified; outputs are
 *    fully overwritten (never accumulated).
 *  - The library performs no device allocation: every device buffer,
 *    including the mesh tables and solver work vectors, lives in workspace
 *    that the caller allocates (e.g. a torch uint8 tensor) and keeps alive
 *    until dg_destroy_mesh / the end of the call that uses it; the one
 *    exception is the built-in per-GPU array of dg_solve_poisson_noalloc.
 *    The mesh handle holds one small pinned host buffer and one event (freed
 *    by dg_destroy_mesh).
 *  - Calls on different mesh handles may run concurrently from different
 *    threads; two solves on one handle must not overlap (the handle caches
 *    eigenvalue estimates and stages the solver's scalars), and a wall-shear
 *    update (dg_update_wall_shear, dg_update_wall_shear_nodes) must not
 *    overlap any other call on its handle: it swaps the handle's current and
 *    previous psi tables and invalidates its inverse-mass cache.
 *
 * Mesh and numbering
 * ------------------
 *  Channel 0<=x<=Lx, -1<=y<=1, 0<=z<=Lz, periodic in x and z, no-slip walls at
 *  y = -1 (optionally displaced to y_w(x) = -1 + wall_amp cos(2 pi x/Lx)) and
 *  y = +1; nx*ny*nz hexahedral cells numbered e = ex + nx (ey + ny ez);
 *  wall-normal vertices y_j = tanh(gamma (2j/ny - 1))/tanh(gamma) (paper
 *  Sec. 5.1; gamma = 0: uniform).  Reference cell [0,1]^3, nodal tensor basis
 *  through the Gauss-Lobatto points, node B = i + (k+1)(j + (k+1) m).
 *  Velocity vector (paper Sec. 3.1, eqs. space/std_fe/enrichment):
 *    [cell][component c=0..2][node B]  followed by the enrichment block
 *    [enriched cell][component][enrichment node], enriched cells being the
 *    wall-adjacent layer of each enriched wall, numbered in increasing cell
 *    index.  Enrichment weights of degree l = 0 (the paper's runs): one
 *    enrichment node, 3 unknowns per enriched cell; l = 1: the eight
 *    trilinear vertex functions N_B = prod_d (b_d ? xi_d : 1 - xi_d),
 *    node bx + 2 (by + 2 bz), 24 unknowns per enriched cell.
 *  Pressure vector: [cell][node B] with degree k_p.
 *  Wall shear stress (tau_w) per wall-face Gauss point of the velocity rule:
 *    [wall w (0 lower, 1 upper)][ez][ex][qz][qx], nq_u^2 values per face.
 */
#ifndef DGWM_H
#define DGWM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  DG_OK = 0,
  DG_ERR_ARG = -1,            /* invalid argument, size or alignment           */
  DG_ERR_WORKSPACE = -2,      /* workspace missing or smaller than required    */
  DG_ERR_HIP = -3,            /* a HIP runtime call failed                     */
  DG_ERR_NONFINITE = -4,      /* NaN/Inf met in a norm or input                */
  DG_ERR_NOT_CONVERGED = -5,  /* solver hit its iteration cap                  */
  DG_ERR_UNSUPPORTED = -6     /* degree/quadrature combination not compiled    */
};

typedef enum { DG_F64 = 0, DG_F32 = 1 } dg_prec;

typedef struct dg_mesh dg_mesh; /* opaque host handle */

typedef struct {
  int32_t nx, ny, nz;     /* cells per direction (ny >= 2 when walls exist)               */
  double Lx, Lz;          /* box lengths in x and z                                      */
  double gamma;           /* tanh grading of the wall-normal vertices (0 = uniform)      */
  double wall_amp;        /* amplitude of the cosine lower wall (0 = flat)               */
  int32_t k_u, k_p;       /* velocity and pressure polynomial degrees                     */
  int32_t nq_u, nq_p;     /* Gauss points per direction: velocity, pressure               */
  int32_t nq_wn;          /* wall-normal Gauss points in enriched cells                   */
  int32_t enrich_lower, enrich_upper; /* enrich the wall-adjacent layer of each wall      */
  int32_t fully_periodic; /* 1: periodic in y as well, no walls, no enrichment (tests)    */
  double nu;              /* kinematic viscosity                                         */
  double kappa, B;        /* Spalding's law constants                                    */
  double ip_factor_u, ip_factor_p; /* multipliers of the (k+1)^2 |F|/|Omega| penalty      */
  double wall_ip_mult;    /* extra penalty factor on no-slip faces (paper: 10)            */
  double theta;           /* adjoint-term sign of the viscous form (+1 symmetric IP)      */
  int32_t psi_kind;       /* enrichment function: DG_PSI_SPALDING or DG_PSI_VANDRIEST     */
  double A_plus;          /* van Driest damping constant A+ (paper: 26)                   */
  double yplus_off;       /* > 0: switch-off threshold of the enrichment (paper: 30), see   */
                          /*      dg_update_wall_shear; 0: the enrichment is always on      */
  int32_t enrich_degree;  /* tensor degree l of the enrichment weights (Sec. 3.1, eq.       */
                          /*   enrichment): 0 or 1.  l = 1 is built for flat walls and, of  */
                          /*   the velocity operators, for dg_apply_velocity_residual,      */
                          /*   dg_apply_convective, dg_eddy_viscosity,                      */
                          /*   dg_apply_viscous_multiscale, dg_apply_inverse_mass,          */
                          /*   dg_solve_helmholtz, dg_apply_pressure_gradient,              */
                          /*   dg_apply_velocity_divergence, dg_divdiv_tau, dg_apply_divdiv, */
                          /*   dg_vorticity_rhs, dg_vorticity, dg_pressure_neumann,         */
                          /*   dg_wall_shear_nodes, dg_project_velocity and                 */
                          /*   dg_dual_splitting_step; dg_projection_step and the batched   */
                          /*   residual return DG_ERR_UNSUPPORTED for it                    */
  int32_t omit_step_tables; /* 1: the mesh workspace leaves out the projection-step tables  */
                          /*   (per-layer spectral factors, enriched-cell couplings), so    */
                          /*   dg_projection_step and dg_dual_splitting_step return         */
                          /*   DG_ERR_UNSUPPORTED on the mesh; 0 (default): reserved         */
} dg_mesh_params;

/* Wall laws for psi = U(y+) (paper Sec. 3.2): Spalding's implicit law with
 * (kappa, B), or van Driest's law (eq. psi) U = int_0^{y+} 2 / (1 + sqrt(1 +
 * (2 kappa s (1 - exp(-s/A+)))^2)) ds, evaluated as in the paper's Appendix A:
 * the integral is tabulated at support points y+_i and the remaining slice
 * [y+_i, y+] is integrated with a 9-point Gauss rule. */
enum { DG_PSI_SPALDING = 0, DG_PSI_VANDRIEST = 1 };

/* ---------------------------------------------------------------- mesh --- */

/* Bytes of device workspace the mesh tables need (>= 0), or a negative
 * DG_ERR_* code if the parameters are invalid or not compiled in. */
int64_t dg_mesh_workspace_bytes(const dg_mesh_params* params);

/* Build the mesh on the current device (paper Sec. 3.1-3.2, 5.1):
 * vertex coordinates, penalties, 1-D basis/quadrature tables, curved-wall
 * geometry at quadrature points, then the enrichment function psi = U(y+),
 * y+ = y_h sqrt(tau_w)/nu, and grad psi at every enriched quadrature point by
 * an FP64 Newton solve of Spalding's law (the law named in Sec. 3.2), and the
 * diagonal of the Poisson operator.
 *   tau_w_host: host array in the tau_w layout above (2*nz*nx*nq_u^2 doubles,
 *               all > 0 and finite), or NULL for tau_w = 1 everywhere.
 *   workspace:  device buffer of at least dg_mesh_workspace_bytes() bytes; it
 *               must stay allocated until dg_destroy_mesh.
 *   out:        receives the handle.  Synchronises `stream` before returning. */
int dg_setup_mesh(const dg_mesh_params* params, const double* tau_w_host, void* workspace, size_t ws_bytes,
                  void* stream, dg_mesh** out);

/* Replace tau_w (device array, tau_w layout, FP64) and recompute psi and grad
 * psi in FP64 (paper Sec. 3.2: the wall shear stress and with it the
 * enrichment space are updated once per time step).  Enqueued on `stream`.
 * Switch-off (paper Sec. 3.2): with yplus_off > 0, the enrichment of an
 * enriched cell is off while every point of its volume rule (nq_u x nq_wn x
 * nq_u) has y+ = y_h sqrt(tau_w)/nu below yplus_off; such a cell gets psi = 0
 * and grad psi = 0, so its enrichment unknowns decouple (their residual rows
 * are zero).  The psi table and activity flags in force before the update
 * are kept as the previous space for dg_project_velocity. */
int dg_update_wall_shear(dg_mesh* mesh, const double* tau_w_dev, void* stream);

/* Nodal wall shear stress of both walls from the FP64 velocity u (paper
 * Sec. 3.2: the wall shear stress is averaged onto the wall nodes with the
 * bilinear (m = 1) hat functions N_B of the wall vertices):
 *   tau_w,B = || int_wall N_B nu (grad u_h) n dA || / int_wall N_B dA,
 * n the outward unit normal (-e_y lower wall, +e_y upper wall), u_h the full
 * velocity including psi u~ with the mesh's current psi, both integrals by
 * the velocity rule's nq_u x nq_u Gauss points of each wall face.
 *   u:         device, dg_num_dofs(mesh, 0) doubles.
 *   tau_nodes: device output, 2*nz*nx doubles in the layout
 *              [wall w (0 lower, 1 upper)][jz][jx], vertex (jx Lx/nx, jz Lz/nz)
 *              of the periodic wall grid; fully overwritten.
 * Deterministic (fixed summation order).  Uses a scratch area of the mesh
 * workspace, so two calls on one handle must not overlap.
 *   Errors: DG_ERR_ARG, DG_ERR_UNSUPPORTED (curved lower wall or a fully
 *   periodic mesh: flat no-slip walls only), DG_ERR_HIP. */
int dg_wall_shear_nodes(const dg_mesh* mesh, const double* u, double* tau_nodes, void* stream);

/* Replace the wall shear stress by a nodal field (device, [wall][jz][jx] as
 * dg_wall_shear_nodes writes it, all > 0 and finite) and recompute psi and
 * grad psi in FP64 (paper Sec. 3.2): tau_w,h is the bilinear interpolation of
 * the nodal values along the wall, constant along the wall normal, and
 * grad y+ = sqrt(tau_w)/nu grad y_h + y_h / (2 nu sqrt(tau_w)) grad tau_w,h.
 * The values are copied; psi entries of points where tau_w,h is not positive
 * and finite become NaN.  The mesh keeps this field until the next
 * dg_update_wall_shear (per-point field) or dg_update_wall_shear_nodes call.
 * Flat no-slip walls only (DG_ERR_UNSUPPORTED otherwise).  Enqueued on
 * `stream`. */
int dg_update_wall_shear_nodes(dg_mesh* mesh, const double* tau_nodes, void* stream);

/* Cell-wise L2 projection of a velocity from the space before the last
 * wall-shear update onto the current one (paper Sec. 3.2, eq. l2):
 *   (v, u_new)_e = (v, u_old)_e  for every v of the current local space,
 * per component and enriched cell, with the enriched cell's quadrature rule;
 * the local space is span{N_B} plus psi_new (l = 0) or the eight psi_new N_B
 * (l = 1, N_B the trilinear vertex functions) while the cell's enrichment is
 * on, the polynomials alone while it is off.  Solved in closed form: with
 * r = phi - P phi (P the L2 projection onto the polynomials, phi the old and
 * the new enrichment functions), the new enrichment coefficients solve
 * (r_new, r_new) u~_new = (r_new, r_old) u~_old (a scalar for l = 0, an 8 x 8
 * Cholesky solve for l = 1) and the polynomial part takes the difference of
 * the two P phi expansions.  Cells without enrichment are copied.  Before any update (or right after setup) this is the identity up
 * to rounding.  Call it once per vector that must follow the new space, after
 * dg_update_wall_shear(_nodes) and before the next update.
 *   u_old, u_new: device, dg_num_dofs(mesh, 0) doubles each.  u_new may be
 *                 u_old: the projection then runs in place and rewrites only
 *                 the enriched cells' entries.
 *   Errors: DG_ERR_ARG, DG_ERR_UNSUPPORTED (curved lower wall), DG_ERR_HIP. */
int dg_project_velocity(const dg_mesh* mesh, const double* u_old, double* u_new, void* stream);

/* Copy the enrichment activity flags (1 on, 0 switched off; see
 * dg_update_wall_shear) of the current space to the device array flags
 * (dg_num_enriched(mesh) int32 values, in enriched-cell order). */
int dg_enrichment_active(const dg_mesh* mesh, int32_t* flags, void* stream);

/* Number of entries of the velocity (field 0, polynomial + enrichment) or
 * pressure (field 1) vector; negative on error. */
int64_t dg_num_dofs(const dg_mesh* mesh, int field);

/* Number of enriched cells. */
int64_t dg_num_enriched(const dg_mesh* mesh);

/* Releases the handle and its pinned host buffer (not the caller's workspace). */
void dg_destroy_mesh(dg_mesh* mesh);

/* ----------------------------------------------------------- operators --- */

/* Velocity residual r = R(u) for every test function (paper Sec. 4.2):
 *   r(phi) = (grad phi, 2 nu eps(u) - u (x) u)_e
 *          + sum_F ( phi . [ {{u (x) u}} n + Lambda/2 (u- - u+)
 *                            - {{2 nu eps(u)}} n + tau_F nu (u- - u+) ]
 *                    - theta nu eps(phi) : ((u- - u+) (x) n) )_F
 * with the local Lax-Friedrichs Lambda = max(2|u-.n|, 2|u+.n|), mirror data
 * u+ = -u-, grad u+ = grad u- and tau_F x wall_ip_mult on no-slip walls,
 * u = u_bar + psi sum_B N^l_B u~_B in enriched cells (test functions N_B e_c
 * and psi N^l_B e_c; l = 0: psi e_c), quadrature nq_u^3 (nq_u x nq_wn x nq_u
 * in enriched cells).  M du/dt = -r.
 *   prec: DG_F64 -> u, r are double*; DG_F32 -> float* (psi tables stay FP64).
 *   u, r: device vectors of dg_num_dofs(mesh, 0) entries; u != r. */
int dg_apply_velocity_residual(const dg_mesh* mesh, dg_prec prec, const void* u, void* r, void* stream);

/* Convective part of the velocity residual, the term F^c_e of the explicit
 * convective step (paper Sec. 4.1 eq. convstep, Sec. 4.2 eq. convstepspat):
 *   r_c(phi) = -(grad phi, u (x) u)_e
 *            + sum_F ( phi . [ {{u (x) u}} n + Lambda/2 (u- - u+) ] )_F,
 * i.e. dg_apply_velocity_residual with nu = 0 (same kernels, local
 * Lax-Friedrichs Lambda, mirror data u+ = -u- on no-slip walls, enriched
 * cells u = u_bar + psi u~).  Arguments and errors as for
 * dg_apply_velocity_residual. */
int dg_apply_convective(const dg_mesh* mesh, dg_prec prec, const void* u, void* r, void* stream);

/* Most meshes one batched call takes. */
#define DG_MAX_BATCH 4096

/* Device workspace (bytes) of a batched velocity call over n meshes, or
 * DG_ERR_ARG when n is outside [1, DG_MAX_BATCH]. */
int64_t dg_batch_workspace_bytes(int32_t n);

/* The velocity residual of paper Sec. 4.2 (as dg_apply_velocity_residual)
 * for n independent meshes in as few launches as there are distinct
 * (degree, quadrature, curved) groups: the cells of every mesh of a group
 * are concatenated into one grid.  Entry i writes r[i] = R_i(u[i]) on
 * meshes[i]; the result is bit-for-bit that of the single-mesh call.  This is
 * the serving path for many small wall-modelled channels (one per request).
 *   meshes, u, r: host arrays of n entries; u[i], r[i] device vectors as for
 *                 the single-mesh call; outputs must be pairwise distinct.
 *   workspace:    device, 256-byte aligned, >= dg_batch_workspace_bytes(n);
 *                 it holds the launch descriptors, so it must not be reused
 *                 before the launches on `stream` have run.
 *   The descriptors go up with one asynchronous copy from pinned staging
 *   owned by the calling thread (8 slots used round-robin, allocated on
 *   first use and kept for the thread's lifetime); the call waits only when
 *   the copy that last used its slot, 8 calls earlier, has not yet run.
 *   Errors: DG_ERR_ARG, DG_ERR_WORKSPACE, DG_ERR_UNSUPPORTED, DG_ERR_HIP. */
int dg_apply_velocity_residual_batched(const dg_mesh* const* meshes, int32_t n, dg_prec prec, const void* const* u,
                                       void* const* r, void* workspace, size_t ws_bytes, void* stream);

/* Inverse of the velocity mass matrix, x = M^{-1} r, so that the
 * semi-discrete momentum balance M du/dt = -R(u) of the residual above (paper
 * Sec. 4.1-4.2) advances explicitly as du/dt = -M^{-1} R(u).  Per cell and
 * component M_ij = (phi_i, phi_j)_e over the cell's local basis (N_B, plus
 * the enrichment functions psi N^l_B in an enriched cell whose enrichment is
 * on; l = 1: a Schur complement on the 8 enrichment rows, the Gram matrix of
 * psi N_B - P(psi N_B)) with the cell's own quadrature
 * rule (nq_u^3; nq_u x nq_wn x nq_u in enriched cells); the enrichment
 * unknowns of a switched-off cell are set to 0.  Block-diagonal (cell-local):
 * regular cells by the tensor product of inverse 1-D mass matrices, enriched
 * cells by the Schur complement on the enrichment row.  The enriched blocks
 * are ill-conditioned where psi is close to a polynomial on the cell (cond
 * 1e6-1e8 at wall-cell tops of y+ 50-400), which bounds the attainable
 * accuracy of any M^{-1} r there.  The first call after setup or after a
 * wall-shear update also fills a per-mesh cache of the enriched cells'
 * polynomial parts of psi on `stream`; a later call on another stream must be
 * ordered after that one.  On the curved-wall mesh (l = 0) a cell's block has
 * no tensor-product inverse (|det J| varies over the cell): each cell runs
 * preconditioned CG on its polynomial block (the tensor inverse of the
 * reference mass matrix over the cell volume as preconditioner, at most 100
 * iterations, to a relative residual of 1e-15), and an enriched cell
 * eliminates its psi row through the Schur complement formed pointwise.
 *   r, x: device, dg_num_dofs(mesh, 0) doubles; x may be r (in place).
 *   Errors: DG_ERR_ARG, DG_ERR_UNSUPPORTED (a degree combination not
 *   compiled), DG_ERR_HIP. */
int dg_apply_inverse_mass(const dg_mesh* mesh, const double* r, double* x, void* stream);

/* Pressure gradient term of the dual-splitting scheme (paper Sec. 4.2):
 *   g(v) = -(div v, p)_e + (v . n, {{p}})_{boundary of e}
 * for every velocity test function v (N_B e_c, and in enriched cells psi e_c
 * for l = 0 or psi N_B e_c over the eight vertex functions for l = 1), {{p}}
 * the central average of the two traces, on no-slip walls the
 * interior value {{p}} = p- (Sec. 4.2, projection step).  Velocity quadrature of the cell (nq_u^3, nq_u x
 * nq_wn x nq_u in enriched cells) and of its faces.  On the curved-wall mesh
 * (l = 0) the geometry enters per point (J^{-1}, |det J| and the curved
 * normals of the isoparametric cells).
 *   p: device, dg_num_dofs(mesh, 1) doubles; g: device, dg_num_dofs(mesh, 0)
 *   doubles (velocity layout, enrichment rows included), distinct from p.
 *   Errors: DG_ERR_ARG, DG_ERR_UNSUPPORTED (a degree combination not
 *   compiled), DG_ERR_HIP. */
int dg_apply_pressure_gradient(const dg_mesh* mesh, const double* p, double* g, void* stream);

/* Velocity divergence term (paper Sec. 4.2):
 *   c(q) = -(grad q, u)_e + (q, {{u}} . n)_{boundary of e}
 * for every pressure test function q, u the full velocity (its enrichment
 * included, for l = 1 the neighbour's four coefficients on a shared face),
 * on no-slip walls the interior value {{u}} = u- (Sec. 4.2, the boundary
 * condition of this term in the pressure Poisson equation); the same
 * quadrature as the gradient, so that q^T C u = -u^T P q wherever the rules
 * integrate div(q u) exactly and q vanishes on the walls.  Curved-wall meshes
 * (l = 0) as for dg_apply_pressure_gradient.
 *   u: device, dg_num_dofs(mesh, 0) doubles; c: device, dg_num_dofs(mesh, 1)
 *   doubles (pressure layout), distinct from u.
 *   Errors: as for dg_apply_pressure_gradient. */
int dg_apply_velocity_divergence(const dg_mesh* mesh, const double* u, double* c, void* stream);

/* Div-div penalty parameter of the projection step (paper Sec. 4.2, eq.
 * tauD), per cell: tau_D,e = ||u||_e h_e dt_over_cr with ||u||_e the volume
 * average of |u| over the cell (u the full velocity, psi u~ included, the
 * cell's velocity rule), h_e the cube root of the cell volume and dt_over_cr
 * the time step over the global Courant number.
 *   u: device, dg_num_dofs(mesh, 0) doubles (the previous step's velocity);
 *   tau_d: device output, nx*ny*nz doubles in cell order.  Curved-wall
 *   meshes (l = 0) take J^{-1} and |det J| per point.
 *   Errors: DG_ERR_ARG, DG_ERR_UNSUPPORTED, DG_ERR_HIP. */
int dg_divdiv_tau(const dg_mesh* mesh, const double* u, double dt_over_cr, double* tau_d, void* stream);

/* Div-div penalty (paper Sec. 4.2, eq. div-div): out(v) = (div v, tau_D,e div u)_e
 * for every velocity test function v (N_B e_c, and the enrichment functions
 * psi e_c (l = 0) or psi N_B e_c (l = 1) in enriched cells), u the full
 * velocity, with the cell's velocity rule; cell-local.
 *   tau_d: device, nx*ny*nz doubles (e.g. from dg_divdiv_tau); u, out:
 *   device, dg_num_dofs(mesh, 0) doubles, distinct.  Curved-wall meshes
 *   (l = 0) take J^{-1} and |det J| per point.
 *   Errors: DG_ERR_ARG, DG_ERR_UNSUPPORTED, DG_ERR_HIP. */
int dg_apply_divdiv(const dg_mesh* mesh, const double* tau_d, const double* u, double* out, void* stream);

/* Element-wise projection step of the dual-splitting scheme (paper Sec. 4.2,
 * eq. projectionspat), cell by cell:
 *   (M_e + D_e) x = M_e u_hat - scale g,
 * M_e the velocity mass matrix and D_e the div-div penalty with tau_d (as in
 * dg_apply_inverse_mass and dg_apply_divdiv), g = P p the pressure gradient
 * term (dg_apply_pressure_gradient; with scale = dt/gamma_0 this is the
 * projection u^ - dt/gamma_0 grad p of the paper's scheme).  Every cell is
 * solved directly (exact up to rounding, no iteration): per distinct cell
 * height the whitened div-div form is diagonalised once, so that a cell's
 * solve is two dense products shared by its layer plus 1-D sweeps; enriched
 * cells add a 3 x 3 Schur complement on the enrichment unknowns.
 * The first call on a mesh computes the per-layer tables on the host and
 * waits for their copy to the device (host-synchronous once; about a second
 * at k_u = 4).  The enriched cells' psi-dependent parts are cached until the
 * next wall-shear update, as for dg_apply_inverse_mass.  A call that fills
 * the tables or the cache writes to the handle: like an update, it must not
 * overlap other calls on the same handle.
 *   tau_d: device, nx*ny*nz doubles; u_hat, g, x: device, dg_num_dofs(mesh,
 *   0) doubles, x distinct from u_hat, g and tau_d.  Flat meshes only.  Fills the
 *   inverse-mass cache on its first call after a wall-shear update (see
 *   dg_apply_inverse_mass).
 *   Errors: DG_ERR_ARG, DG_ERR_UNSUPPORTED, DG_ERR_HIP, DG_ERR_NOT_CONVERGED
 *   (a table's eigendecomposition did not converge). */
int dg_projection_step(const dg_mesh* mesh, const double* tau_d, const double* u_hat, const double* g, double scale,
                       double* x, void* stream);

/* Points of the eddy-viscosity table: dg_num_enriched(mesh) times the points
 * of one enriched cell (its volume rule nq_u x nq_wn x nq_u, x fastest, then
 * the face rules of its faces x=0, x=1, y=0, y=1, z=0, z=1), or a negative
 * DG_ERR_* code. */
int64_t dg_eddy_viscosity_points(const dg_mesh* mesh);

/* Eddy viscosity of the RANS scale (paper Sec. 2.2) at every quadrature point
 * of the enriched cells, from the enrichment coefficients of u (u~ = psi ut,
 * l = 0, so grad u~ = ut (x) grad psi; l = 1: grad u~ = sum_B ut_B (x)
 * (N_B grad psi + psi grad N_B)):
 *   nu_t = l_mix^2 |eps(u~)|,  |eps| = sqrt(2 eps : eps)             (eq. mix)
 *   l_mix = kappa y_DES (1 - exp(-y+/A+))                            (eq. lmix)
 *   y_DES = (y^-beta + (c_des h)^-beta)^(-1/beta), 0 at the wall     (eq. ydes)
 * with y the wall distance, y+ = y sqrt(tau_w)/nu, h the wall-normal cell
 * width over k_u + 1, kappa and A+ the mesh's constants and the psi table in
 * force.  The paper's values are c_des = 0.85 and beta = 6.  Switched-off
 * cells get 0.  Flat walls only.
 *   u:   device, dg_num_dofs(mesh, 0) doubles (only its enrichment block is read);
 *   nut: device output, dg_eddy_viscosity_points(mesh) doubles, layout
 *        [enriched cell][point] as described there.
 *   Errors: DG_ERR_ARG, DG_ERR_UNSUPPORTED (curved wall), DG_ERR_HIP. */
int dg_eddy_viscosity(const dg_mesh* mesh, const double* u, double c_des, double beta, double* nut, void* stream);

/* Viscous term of the multiscale method (paper Sec. 4.2, eq.
 * viscous_multiscale): out(v) = -F^nu_e(v_bar, v~, u_bar, u~) for every test
 * function v (v_bar = N_B e_c; v~ = psi N^l_B e_c in enriched cells), with
 * F^a(w) = 2 a eps(w), the four row blocks and face-class masks of the
 * equation (adjoint sign -1):
 *   volume:    (eps(v_bar), F^nu(u_bar) + F^nuhat(u~)) + (eps(v~), F^{nu+nu_t}(u~)),
 *              nuhat = min(nu + nu_t, 2 sqrt(nu (nu + nu_t)))  (Sec. 4.3, eq. minvt);
 *   faces without an enriched side (the SIP form of the velocity residual
 *              with theta = -1): (F^nu(v_bar)/2, [u_bar] (x) n)
 *              - (v_bar, {{F^nu(u_bar)}} n) + (v_bar, tau nu [u_bar]);
 *   interface faces (one enriched side): (F^nu(v_bar)/2, [u] (x) n)
 *              - (v, {{F^nu(u_bar)}} n) + (v, tau nu [u]), the adjoint part for
 *              v_bar only;
 *   faces of an enriched cell whose other side is enriched or a wall:
 *              (F^nu(v_bar)/2, [u_bar] (x) n) - (v_bar, {{F^nu(u_bar)}} n)
 *              - (v, {{F^{nu+nu_t}(u~)}}_w n) + (v, tau nu [u]), plus
 *              (w- F^{nu+nu_t}(v~), [u] (x) n) for v~,
 * u = u_bar + u~, {{.}}_w the harmonic weights of eq. harmweights, mirror data
 * on walls (u+ = -u-, grad u+ = grad u-, nu_t+ = nu_t-), tau as in
 * dg_apply_velocity_residual (x wall_ip_mult on walls), velocity quadrature
 * (R9/R10 rules of the residual).  Linear in u for the given nu_t; the
 * Helmholtz step of the paper's scheme is (gamma_0/dt) M u + A u = rhs.
 *   nut: device, from dg_eddy_viscosity (may be NULL without enriched cells);
 *   u, out: device, dg_num_dofs(mesh, 0) doubles, distinct.  FP64, flat walls.
 *   Errors: DG_ERR_ARG, DG_ERR_UNSUPPORTED, DG_ERR_HIP. */
int dg_apply_viscous_multiscale(const dg_mesh* mesh, const double* nut, const double* u, double* out, void* stream);

/* Right-hand side of the vorticity projection (paper Sec. 4.2: the
 * vorticity omega_h of the pressure Neumann data is precomputed by L2
 * projection onto the velocity space):
 *   b(v) = (v, curl u)_e
 * for every velocity test function (N_B e_c, and psi e_c in enriched cells),
 * u = u_bar + psi u~ (so curl u includes grad psi x u~), the cell's velocity
 * rule (nq_u^3; nq_u x nq_wn x nq_u in enriched cells).
 *   u, b: device, dg_num_dofs(mesh, 0) doubles, distinct.  On the
 *   curved-wall mesh (l = 0) grad u = J^{-T} grad_xi u and |det J| enter
 *   per point.
 *   Errors: DG_ERR_ARG, DG_ERR_UNSUPPORTED, DG_ERR_HIP. */
int dg_vorticity_rhs(const dg_mesh* mesh, const double* u, double* b, void* stream);

/* omega = M^{-1} b with b from dg_vorticity_rhs: the L2 projection of curl u
 * onto the enriched velocity space (the inverse mass matrix of
 * dg_apply_inverse_mass; on the curved-wall mesh its per-cell CG).  u,
 * omega: distinct device vectors. */
int dg_vorticity(const dg_mesh* mesh, const double* u, double* omega, void* stream);

/* Wall term of the pressure equation with the high-order Neumann data (paper
 * Sec. 4.1 eq. bc_d_pres, the wall flux of eq. ipflux), ADDED into rhs:
 *   rhs(q) += int_wall q h_N dA,
 *   h_N = -( sum_i beta[i] (div(u_i (x) u_i) + nu curl omega_i) - f ) . n
 * for the nhist (1 or 2) previous velocities u_i and their vorticities
 * omega_i (dg_vorticity), n the outward wall normal (-e_y lower, +e_y upper
 * wall; on the curved-wall mesh, l = 0, the normal of the isoparametric wall,
 * +-|det J| J^{-T} e_y normalised, with all three flux components),
 * evaluated at the Gauss points of the velocity face rule (nq_u x
 * nq_u) with u = u_bar + psi u~ (psi vanishes on the wall, grad psi does not)
 * and tested with the pressure basis; only the wall cells' pressure rows
 * change.  Nothing is added on a fully periodic box.
 *   u, omega: host arrays of nhist device vectors (velocity layout);
 *   beta: host, nhist extrapolation weights; f: host, body force (3
 *   doubles, or NULL for none); rhs: device, dg_num_dofs(mesh, 1) doubles.
 *   Errors: DG_ERR_ARG, DG_ERR_UNSUPPORTED (curved wall), DG_ERR_HIP. */
int dg_pressure_neumann(const dg_mesh* mesh, int32_t nhist, const double* const* u, const double* const* omega,
                        const double* beta, const double* f, double* rhs, void* stream);

/* Restarted GMRES parameters and statistics of the Helmholtz step. */
typedef struct {
  double rtol;          /* stop when ||gamma b - H x||_2 <= rtol ||gamma b||_2 (true residual, see below) */
  int32_t max_iter;     /* cap on the Arnoldi steps over all restart cycles                           */
  int32_t restart;      /* Krylov vectors per cycle, 1..100                                           */
} dg_gmres_params;

typedef struct {
  int32_t iterations, restarts;
  double rel_resid;     /* final ||gamma b - H x|| / ||gamma b||                                       */
  double seconds;       /* host wall time of the call                                                  */
} dg_gmres_stats;

/* Device workspace of dg_solve_helmholtz: restart + 1 velocity vectors plus
 * scalars, or a negative DG_ERR_* code. */
int64_t dg_helmholtz_workspace_bytes(const dg_mesh* mesh, const dg_gmres_params* gp);

/* Helmholtz step of the dual-splitting scheme (paper Sec. 4.1 eq. visc,
 * Sec. 4.2 eq. helmholtzspat):
 *   (gamma0/dt) M x + A x = (gamma0/dt) M b,
 * A the multiscale viscous operator of dg_apply_viscous_multiscale with the
 * eddy viscosity nut (adjoint sign -1, so A is not symmetric), M the
 * velocity mass matrix, b the second intermediate velocity u_hathat.  Solved
 * as H x = gamma x + M^{-1} A x = gamma b (gamma = gamma0/dt) by restarted
 * GMRES in FP64 (the paper solves this step with GMRES, Sec. 5.1): the
 * cell-wise M^{-1} of dg_apply_inverse_mass is the left preconditioner, and
 * the residual is measured in that preconditioned form.  The Arnoldi
 * process runs on M^{-1} A (the same Krylov spaces; gamma is added to the
 * Hessenberg diagonal), orthogonalised by classical Gram-Schmidt applied
 * twice with the second pass delayed into the next step (two passes over
 * the basis per step); the projections stay on the device, one host
 * read-back per Arnoldi step, deterministic reductions; convergence is
 * confirmed with the true residual.
 *   nut: device, from dg_eddy_viscosity (may be NULL without enriched cells);
 *   b, x: device, dg_num_dofs(mesh, 0) doubles, distinct; x holds the
 *   initial guess (e.g. b); ws: device, 256-byte aligned, >= dg_helmholtz_workspace_bytes.
 *   Errors: DG_ERR_ARG, DG_ERR_WORKSPACE, DG_ERR_UNSUPPORTED (curved wall),
 *   DG_ERR_NONFINITE, DG_ERR_NOT_CONVERGED (stats filled), DG_ERR_HIP. */
int dg_solve_helmholtz(const dg_mesh* mesh, const double* nut, double gamma0_over_dt, const double* b, double* x,
                       const dg_gmres_params* gp, void* ws, size_t ws_bytes, dg_gmres_stats* stats, void* stream);

/* SIP Poisson operator y = A p, A = -L of paper Sec. 4.2 (pressure Laplace
 * term, flux eq. ipflux) with homogeneous Neumann data on the walls:
 *   (A p)(q) = sum_e (grad q, grad p)_e + sum_{interior F} [ -1/2 (grad q.n)(p- - p+)
 *              - q ({{grad p}}.n - tau_F (p- - p+)) ]_F,
 * tau_F = ip_factor_p (k_p+1)^2 max(|F|/|Omega-|, |F|/|Omega+|), nq_p^3 Gauss
 * points.  Flat (box) meshes only.  p, y: device vectors of
 * dg_num_dofs(mesh, 1) entries of the precision's type; p != y. */
int dg_apply_poisson(const dg_mesh* mesh, dg_prec prec, const void* p, void* y, void* stream);

/* Diagonal of the Poisson operator (FP64, computed at setup) copied to the
 * device vector d (dg_num_dofs(mesh, 1) doubles). */
int dg_poisson_diagonal(const dg_mesh* mesh, double* d, void* stream);

/* Levels of the geometric multigrid hierarchy of the pressure space (the
 * preconditioner of dg_solve_poisson with multigrid = 1; Sec. 4.4 names
 * multigrid-preconditioned CG as the paper's pressure solver).  Level 0 is
 * the mesh; level l+1 merges cell pairs of level l along every direction
 * with an even cell count (y only while at least 4 layers remain, 2 when
 * fully periodic) until the dense coarse solve is small enough.  Writes six
 * int32 per level for the first min(levels, cap) levels: nx, ny, nz, cx,
 * cy, cz (cx, cy, cz = 1 where level l was coarsened from l-1 along x, y, z;
 * zero on level 0).  out may be NULL when cap is 0.  Returns the number of
 * levels (0 on curved meshes, which have no hierarchy) or a negative error
 * code. */
int dg_mg_levels(const dg_mesh* mesh, int32_t* out, int32_t cap);

/* One transfer between levels l and l+1 of that hierarchy, queued on
 * stream.  The prolongation P is the exact embedding of the level-(l+1) DG
 * space into the level-l one: nodal values of each coarse-cell polynomial
 * at the Gauss-Lobatto nodes of its 2, 4 or 8 child cells (a y pair split
 * at the ratio of the two layer heights).  Vectors use the pressure layout
 * of the level (cells x fastest, then y, z; nodes (k_p+1)^3 per cell, x
 * fastest).
 *   direction 0 (restriction): out = P^T in; in: level l, out: level l+1.
 *   direction 1 (prolongation): out = add + P in; in: level l+1, add and
 *     out: level l (add may equal out; pass a zero vector to get P in).
 *   prec: DG_F64 -> double vectors, DG_F32 -> float.  in must not alias out.
 * Errors: DG_ERR_ARG for a level outside 0 .. levels-2, an unknown
 * direction or precision, or NULL pointers; DG_ERR_UNSUPPORTED on curved
 * meshes. */
int dg_mg_transfer(const dg_mesh* mesh, int32_t level, int32_t direction, dg_prec prec, const void* in,
                   const void* add, void* out, void* stream);

/* ---------------------------------------------------------------- solve --- */

typedef struct {
  double rtol;          /* stop when ||b - A x||_2 <= rtol ||b||_2 (e.g. 1e-10), true residual  */
  int32_t max_outer;    /* cap on the FP64 (outer) conjugate-gradient iterations                */
  int32_t max_inner;    /* mixed: FP32 CG iterations per preconditioner call (0: polynomial only)*/
  int32_t cheb_degree;  /* degree of the Jacobi-Chebyshev polynomial preconditioner (>= 1)      */
  int32_t mixed;        /* 1: preconditioner in FP32; 0: everything FP64                        */
  int32_t multigrid;    /* 1: the preconditioner is one geometric multigrid V-cycle whose        */
                        /*    smoother is the degree-cheb_degree Jacobi-Chebyshev polynomial;    */
                        /*    0: the polynomial alone (or the inner CG, see max_inner)           */
  int32_t coarse_degree;/* multigrid: smoother degree on the levels below the finest           */
                        /*    (0: cheb_degree; otherwise >= 1)                                   */
} dg_solve_params;

typedef struct {
  int32_t outer_its, inner_its_total;
  int32_t op_applies_f64, op_applies_f32;
  double rel_resid;     /* final ||b - A x|| / ||b|| in FP64                              */
  double seconds;       /* host wall time of the call                                     */
} dg_solve_stats;

/* Bytes of device workspace dg_solve_poisson needs. */
int64_t dg_solve_workspace_bytes(const dg_mesh* mesh, const dg_solve_params* sp);

/* The same size computed from mesh parameters before any mesh exists (for
 * admission by device-memory footprint); DG_ERR_ARG on invalid parameters. */
int64_t dg_solve_workspace_bytes_for(const dg_mesh_params* params, const dg_solve_params* sp);

/* Solve A x = b for the singular SIP Poisson operator (null space: constants;
 * the pressure equation of the paper's dual-splitting step, Sec. 4.1-4.2).
 * b is projected to zero mean first (the compatibility condition); x is
 * returned with zero mean.  x holds the initial guess on entry.
 * Outer loop: flexible preconditioned CG in FP64 (residuals, norms and dot
 * products always FP64, deterministic fixed-order reductions, true residual
 * recomputed periodically and before convergence is accepted).
 * Preconditioner (the paper's solver is multigrid-preconditioned CG, Sec. 4.4):
 *   multigrid = 1: one V-cycle over the mesh's nested h-levels (cell pairs
 *     merged along every direction with an even count), smoothing by the
 *     Chebyshev polynomial in D^{-1} A_l on [lmax_l/20, 1.1 lmax_l] of degree
 *     cheb_degree on the finest level and coarse_degree below it, transfers
 *     by the exact embedding of the coarse DG space and its transpose, the
 *     coarsest level by a dense pseudo-inverse; max_inner is ignored;
 *   multigrid = 0: the Chebyshev polynomial on [lmax/30, 1.1 lmax] alone,
 *     optionally wrapped in max_inner FP32 CG iterations.
 * lmax of each level comes from 20 Lanczos steps and is cached in the mesh.
 * With mixed = 1 the preconditioner runs in FP32 on the normalised residual.
 * Reads back one scalar per outer iteration (the next preconditioner
 * application is queued before the host waits for it) and returns when
 * converged.
 *   b, x: device double vectors; workspace: dg_solve_workspace_bytes().
 *   Errors: DG_ERR_NOT_CONVERGED (stats filled) after max_outer iterations,
 *   DG_ERR_NONFINITE on NaN/Inf. */
int dg_solve_poisson(const dg_mesh* mesh, const dg_solve_params* sp, const double* b, double* x, void* workspace,
                     size_t ws_bytes, dg_solve_stats* stats, void* stream);

/* Bytes of solver workspace dg_solve_poisson_noalloc holds per GPU (64 MiB:
 * Poisson meshes up to about 550,000 unknowns, e.g. 16^3 cells at k_p = 4). */
#define DG_NOALLOC_SOLVE_MAX_BYTES ((size_t)64 << 20)

/* dg_solve_poisson without a workspace argument, for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  Same solve, same arguments and results
 * as dg_solve_poisson (bit for bit on the same inputs); the solver's work
 * vectors and partial sums live in a device array of
 * DG_NOALLOC_SOLVE_MAX_BYTES built into the library, one per GPU, held until
 * the process ends.  The call allocates nothing (no hipMalloc / hipFree or
 * allocating library routine); its first call on a device resolves that
 * device's array address once.  Every call on one GPU shares its array and
 * leaves its last contents there (each solve writes every byte it reads), so
 * calls that overlap on one GPU, from any thread or stream, race: serialise
 * them.  The mesh must live on the current device.
 *   Errors: as dg_solve_poisson, plus DG_ERR_WORKSPACE when
 *   dg_solve_workspace_bytes(mesh) exceeds DG_NOALLOC_SOLVE_MAX_BYTES. */
int dg_solve_poisson_noalloc(const dg_mesh* mesh, const dg_solve_params* sp, const double* b, double* x,
                             dg_solve_stats* stats, void* stream);

/* Device bytes of the workspace of a batched solve over these n meshes
 * with these parameters, or a negative DG_ERR_* code. */
int64_t dg_solve_batch_workspace_bytes(const dg_mesh* const* meshes, int32_t n, const dg_solve_params* sp);

/* The solves of n independent meshes (the serving path: one pressure step,
 * Sec. 4.1 eq. poisson, per wall-modelled channel) advanced together: every
 * outer iteration of every unconverged mesh runs in the same launches, one
 * per step of the iteration and degree group (operator applications and
 * fused Chebyshev steps of every multigrid level, transfers, coarse solves,
 * vector updates and reductions), from descriptor tables kept in batch_ws
 * while the set of unconverged meshes is unchanged.  A mesh leaves the batch
 * when it converges.  Per mesh the method and the stopping rule are those of
 * dg_solve_poisson with multigrid = 1, step by step with the same kernel
 * bodies and reduction layout (a block count set by the vector length): a
 * mesh gets bit-for-bit the x and statistics of dg_solve_poisson, in any
 * batch.  Descriptors travel in kernel
 * arguments (up to 8 to 32 meshes per launch; larger batches take several).
 * Eigenvalue estimates missing from a mesh's cache are computed for all such
 * meshes together at the start.  One host read-back per outer
 * iteration for the whole batch, through pinned memory owned by the calling
 * thread (allocated on its first call and kept for the thread's lifetime).
 *   meshes, b, x, ws, ws_bytes: host arrays of n entries; b[i], x[i] device
 *     vectors of dg_num_dofs(meshes[i], 1) doubles (x[i] holds the initial
 *     guess), ws[i] a workspace of ws_bytes[i] >= dg_solve_workspace_bytes
 *     bytes, all pairwise distinct;
 *   sp: shared parameters (multigrid must be 1);
 *   stats, codes: host arrays of n entries (may be NULL): per mesh
 *     statistics and status (DG_OK, DG_ERR_NOT_CONVERGED, DG_ERR_NONFINITE);
 *   batch_ws: device, >= dg_solve_batch_workspace_bytes(meshes, n, sp)
 *     (one row of read-back scalars per mesh).
 * Returns DG_OK when the batch ran (per mesh outcomes in codes), else
 * DG_ERR_ARG, DG_ERR_WORKSPACE, DG_ERR_UNSUPPORTED (multigrid = 0, a curved
 * mesh or one without a coarser level) or DG_ERR_HIP.  Calls on one thread
 * must not overlap (they share its pinned read-back rows); the call returns after
 * the stream has drained. */
int dg_solve_poisson_batched(const dg_mesh* const* meshes, int32_t n, const dg_solve_params* sp,
                             const double* const* b, double* const* x, void* const* ws, const size_t* ws_bytes,
                             dg_solve_stats* stats, int32_t* codes, void* batch_ws, size_t batch_ws_bytes,
                             void* stream);

/* ------------------------------------------------- dual-splitting step --- */

typedef struct {
  double dt;             /* time step                                                            */
  double gamma0;         /* BDF coefficient of the new level (BDF2: 3/2; BDF1: 1)                */
  double alpha[2];       /* coefficients of u^n, u^{n-1} (BDF2: 2, -1/2; BDF1: 1, 0)             */
  double beta[2];        /* extrapolation of F^c and of the Neumann data (EXT2: 2, -1; 1, 0)    */
  int32_t order;         /* time levels J = 1 or 2                                               */
  double f[3];           /* constant body force (e.g. the channel's driving pressure gradient)   */
  double dt_over_cr;     /* div-div penalty parameter dt/Cr of eq. tauD                          */
  double c_des, beta_des;/* eddy viscosity constants of eq. ydes (paper: 0.85, 6)                */
  dg_solve_params poisson;
  dg_gmres_params helmholtz;
} dg_step_params;

typedef struct {
  dg_solve_stats poisson;
  dg_gmres_stats helmholtz;
  double seconds;        /* host wall time of the step                                           */
  int32_t projection_its;/* l = 1: GMRES iterations of the projection step (l = 0: 0, solved directly) */
} dg_step_stats;

/* Device workspace of dg_dual_splitting_step (7 velocity vectors, the
 * pressure right-hand side, tau_D, nu_t, the Poisson and Helmholtz solver
 * workspaces), or a negative DG_ERR_* code. */
int64_t dg_step_workspace_bytes(const dg_mesh* mesh, const dg_step_params* sp);

/* One time step of the dual-splitting scheme (paper Sec. 4.1; element-wise
 * forms of Sec. 4.2), every operator on the GPU:
 *   1 convective step (eq. convstepspat):
 *       u^ = (sum_i alpha_i u^{n-i} - dt M^{-1} sum_i beta_i F^c(u^{n-i})) / gamma0 + dt/gamma0 f
 *   2 pressure (eq. poissonspat with eq. ipflux on the walls): A p = -(gamma0/dt) C u^
 *       + int_wall q h_N, h_N the high-order Neumann data of eq. bc_d_pres from u^{n-i} and
 *       their projected vorticities; solved by dg_solve_poisson with sp->poisson (p holds the
 *       initial guess on entry, e.g. the previous pressure, and the zero-mean p^{n+1} on exit)
 *   3 projection (eq. projectionspat): (M + D) u^^ = M u^ - dt/gamma0 P p, tau_D from u^n;
 *       solved directly for l = 0 (dg_projection_step) and, for l = 1, as the block-diagonal
 *       u^^ + M^{-1} D u^^ = u^ - dt/gamma0 M^{-1} P p by the GMRES of step 4 (relative
 *       residual 1e-12, at most 50000 iterations, sp->helmholtz's restart, from u^; the
 *       near-singular l = 1 mass blocks make this iteration long)
 *   4 Helmholtz (eq. helmholtzspat): (gamma0/dt) M u + A(nu_t) u = (gamma0/dt) M u^^ by
 *       dg_solve_helmholtz with sp->helmholtz, nu_t from the enrichment of u^n, from u^^
 * The wall shear stress and psi are those of the mesh (a caller refreshes them between
 * steps with dg_wall_shear_nodes / dg_update_wall_shear_nodes / dg_project_velocity).
 *   u_n, u_nm1 (order 2 only), u_np1: device velocity vectors, u_np1 distinct from both;
 *   p: device pressure vector; ws: >= dg_step_workspace_bytes.
 *   Errors: those of the steps (DG_ERR_NOT_CONVERGED from either solver, stats filled),
 *   DG_ERR_ARG, DG_ERR_WORKSPACE, DG_ERR_UNSUPPORTED (curved wall), DG_ERR_HIP. */
int dg_dual_splitting_step(const dg_mesh* mesh, const dg_step_params* sp, const double* u_n, const double* u_nm1,
                           double* u_np1, double* p, void* ws, size_t ws_bytes, dg_step_stats* stats, void* stream);

/* ---------------------------------------------------------------- misc --- */

const char* dg_last_error(void);

/* Degree / quadrature combinations compiled into the library, as text. */
const char* dg_build_info(void);

#ifdef __cplusplus
}
#endif

#endif /* DGWM_H */
