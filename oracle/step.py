"""Steps of the dual-splitting scheme (arXiv 1705.08813, Sec. 4.1 eqs.
convstep, poisson, bc_d_pres, visc; Sec. 4.2 eqs. convstepspat, poissonspat,
projectionspat, helmholtzspat), composed from the oracle's operators.

TEST INFRASTRUCTURE ONLY (never used by the product).

Library solvers serve as the solution steps: SciPy's GMRES for the
Helmholtz equation, NumPy's dense least squares for the singular pressure
equation on small meshes.  The vorticity right-hand side and the Neumann
wall term also take the curved-wall mesh (l = 0); the rest is for flat
(box) meshes.
"""
from __future__ import annotations

import numpy as np

from . import (cell_jacobians, enriched_cells, enrichment_active, gauss, gauss_lobatto, lagrange, psi_point,
               psi_volume, psi_volume4, vertex_eta, viscous_multiscale)
from .project import inverse_mass, mass_apply


def _psi(cfg, tau):
    cells = enriched_cells(cfg)
    return psi_volume(cfg, cells, tau=tau) if cells.size else np.zeros((0, 1))


def helmholtz_solve(cfg, u_nut, tau, gamma, b, rtol=1e-11, x0=None):
    """x with gamma M x + A x = gamma M b (Sec. 4.2 eq. helmholtzspat,
    gamma = gamma0/dt, A = -F^nu of eq. viscous_multiscale with nu_t from
    the enrichment of u_nut), by GMRES on the M^{-1}-scaled form
    gamma x + M^{-1} A x = gamma b.  Returns (x, GMRES iterations)."""
    import scipy.sparse.linalg as sla
    psi = _psi(cfg, tau)
    n = cfg.n_vel
    u_nut = np.zeros(n) if u_nut is None else np.asarray(u_nut, dtype=np.float64)   # nu_t stays fixed

    def H(x):
        return gamma * x + inverse_mass(cfg, viscous_multiscale(cfg, x, u_nut=u_nut, tau=tau), psi)

    op = sla.LinearOperator((n, n), matvec=H, dtype=np.float64)
    its = [0]

    def cb(_):
        its[0] += 1

    x, info = sla.gmres(op, gamma * np.asarray(b, dtype=np.float64), x0=b if x0 is None else x0, rtol=rtol, atol=0.0,
                        restart=150, maxiter=8, callback=cb, callback_type="pr_norm")
    if info != 0:
        raise RuntimeError(f"oracle GMRES did not converge: {info}")
    return x, its[0]


def helmholtz_residual(cfg, u_nut, tau, gamma, b, x):
    """gamma M x + A x - gamma M b with the forward mass matrix (no inverse)."""
    psi = _psi(cfg, tau)
    u_nut = np.zeros(cfg.n_vel) if u_nut is None else u_nut
    return gamma * mass_apply(cfg, x, psi) + viscous_multiscale(cfg, x, u_nut=u_nut, tau=tau) \
        - gamma * mass_apply(cfg, b, psi)


# ---------------------------------------------------------------------------
# Vorticity and the high-order pressure Neumann data (Sec. 4.1 eq. bc_d_pres;
# Sec. 4.2 eq. ipflux on the walls)
# ---------------------------------------------------------------------------

def _enr_weights(pts, h, ut):
    """The enrichment weights sum_B N^l_B ut[c][B] at the points and their
    gradients (Sec. 3.1 eq. enrichment): constants for l = 0, trilinear for
    l = 1.  Returns (npts, 3) and (npts, 3, 3) [q, component, direction]."""
    ut = np.asarray(ut, dtype=np.float64)
    nle = ut.size // 3
    U = ut.reshape(3, nle)
    if nle == 1:
        return np.repeat(U.T, len(pts), axis=0), np.zeros((len(pts), 3, 3))
    from .project import _vertex_grads
    N, dN = _vertex_grads(pts, h)
    return N @ U.T, np.einsum("qbd,cb->qcd", dN, U)


def _cell_grads(cfg, u, e, pts, h, psi4_k, ut):
    """Values (npts, 3) and gradients (npts, 3, 3) [q, component, direction]
    of the velocity-space field u on cell e at reference points, the
    enrichment psi sum_B N^l_B u~_B included when psi4_k (psi and grad psi at
    the points) is given (ut: the cell's 3 (l = 0) or 24 (l = 1) coefficients,
    [c][B])."""
    from .project import basis_at, _basis_grad_at
    n3 = (cfg.k_u + 1) ** 3
    U = np.asarray(u[e * 3 * n3:(e + 1) * 3 * n3], dtype=np.float64).reshape(3, n3)
    V = basis_at(cfg, pts)
    G = _basis_grad_at(cfg, pts, h)
    val = V @ U.T
    grad = np.einsum("qbd,cb->qcd", G, U)
    if psi4_k is not None:
        L, dL = _enr_weights(pts, h, ut)
        val += psi4_k[:, 0:1] * L
        grad += L[:, :, None] * psi4_k[:, None, 1:4] + psi4_k[:, 0, None, None] * dL
    return V, val, grad


def _curl(grad):
    return np.stack([grad[:, 2, 1] - grad[:, 1, 2], grad[:, 0, 2] - grad[:, 2, 0], grad[:, 1, 0] - grad[:, 0, 1]], 1)


def vorticity_rhs(cfg, u, tau):
    """b(v) = (v, curl u)_e for every velocity test function (N_B e_c, and the
    enrichment functions psi N^l_B e_c of an enriched cell whose enrichment is
    on) with the cell's velocity rule (nq_u^3, or nq_u x nq_wn x nq_u),
    u = u_bar + psi sum_B N^l_B u~_B.  On the curved-wall mesh (l = 0) the
    gradients and |det J| of the isoparametric map enter point by point."""
    from .project import volume_rule, _nle, _vertex_grads
    nle = _nle(cfg)
    n3 = (cfg.k_u + 1) ** 3
    u = np.asarray(u, dtype=np.float64)
    b = np.zeros(cfg.n_vel)
    eta = vertex_eta(cfg)
    hx, hz = cfg.Lx / cfg.nx, cfg.Lz / cfg.nz
    off = cfg.ncell * 3 * n3
    ecells = enriched_cells(cfg)
    enr = {int(e): k for k, e in enumerate(ecells)}
    psi4 = psi_volume4(cfg, ecells, tau=tau) if ecells.size else None
    pts_e, wts_e = volume_rule(cfg)
    pts_r, wts_r = volume_rule(cfg.with_(nq_wn=cfg.nq_u))
    curved = cfg.wall_amp != 0.0
    if curved and nle != 1:
        raise ValueError("curved meshes: l = 0 only")
    for e in range(cfg.ncell):
        ey = (e // cfg.nx) % cfg.ny
        h = (hx, eta[ey + 1] - eta[ey], hz)
        k = enr.get(e)
        pts, wts = (pts_e, wts_e) if k is not None else (pts_r, wts_r)
        p4 = psi4[k] if k is not None else None
        ut = u[off + 3 * nle * k:off + 3 * nle * (k + 1)] if k is not None else None
        if curved:
            # isoparametric cell: grad N = J^{-T} grad_xi N and w |det J| point by point
            from .project import basis_at, _basis_grad_at
            J = cell_jacobians(cfg, e, pts)
            Ji = np.linalg.inv(J)                                                  # [q][a][d] = dxi_a / dx_d
            G = np.einsum("qba,qad->qbd", _basis_grad_at(cfg, pts, (1.0, 1.0, 1.0)), Ji)
            V = basis_at(cfg, pts)
            grad = np.einsum("qbd,cb->qcd", G, u[e * 3 * n3:(e + 1) * 3 * n3].reshape(3, n3))
            if p4 is not None:
                grad += ut[None, :, None] * p4[:, None, 1:4]                      # grad (psi u~_c) = u~_c grad psi
            cw = _curl(grad) * (wts * np.abs(np.linalg.det(J)))[:, None]
        else:
            V, _, grad = _cell_grads(cfg, u, e, pts, h, p4, ut)
            cw = _curl(grad) * (wts * h[0] * h[1] * h[2])[:, None]
        b[e * 3 * n3:(e + 1) * 3 * n3] = (V.T @ cw).T.reshape(-1)
        if k is not None:
            phi = p4[:, 0:1] * (_vertex_grads(pts, h)[0] if nle == 8 else np.ones((len(pts), 1)))   # (npts, nle)
            b[off + 3 * nle * k:off + 3 * nle * (k + 1)] = (phi.T @ cw).T.reshape(-1)              # [c][B]
    return b


def vorticity(cfg, u, tau):
    """omega_h = L2 projection of curl u_h onto the enriched velocity space
    (Sec. 4.2, below eq. ipflux): M omega = vorticity_rhs."""
    return inverse_mass(cfg, vorticity_rhs(cfg, u, tau), _psi(cfg, tau))


def pressure_neumann(cfg, us, omegas, betas, f, tau):
    """Wall term of the pressure equation with the high-order Neumann data of
    eq. bc_d_pres:  rhs(q) = int_wall q h_N dA,
      h_N = -( sum_i beta_i (div F^c(u_i) + nu curl omega_i) - f ) . n,
    div F^c(u) = div(u (x) u), n the outward normal (-e_y on the lower wall,
    +e_y on the upper one), at the Gauss points of the velocity face rule
    (nq_u x nq_u) against the pressure basis; u_i = u_bar + psi sum_B N^l_B u~_B
    and omega_i likewise in enriched cells (psi = 0 on the wall, grad psi not).
    On the curved-wall mesh (l = 0) n is the normal of the isoparametric wall
    and every component of the flux enters."""
    from .project import _nle
    nle = _nle(cfg)
    if cfg.fully_periodic:
        return np.zeros(cfg.n_p)
    npu, npp = cfg.k_u + 1, cfg.k_p + 1
    n3, p3 = npu ** 3, npp ** 3
    off = cfg.ncell * 3 * n3
    nodes_u, nodes_p = gauss_lobatto(npu), gauss_lobatto(npp)
    gq, gw = gauss(cfg.nq_u)
    eta = vertex_eta(cfg)
    hx, hz = cfg.Lx / cfg.nx, cfg.Lz / cfg.nz
    enr = {int(e): k for k, e in enumerate(enriched_cells(cfg))}
    act = enrichment_active(cfg, tau=tau) if enr else None
    rhs = np.zeros(cfg.n_p)
    for ey, s, sg in ((0, 0.0, -1.0), (cfg.ny - 1, 1.0, 1.0)):
        for ez in range(cfg.nz):
            for ex in range(cfg.nx):
                e = ex + cfg.nx * (ey + cfg.ny * ez)
                h = (hx, eta[ey + 1] - eta[ey], hz)
                k = enr.get(e)
                pts = np.array([(gq[a], s, gq[c]) for c in range(cfg.nq_u) for a in range(cfg.nq_u)])
                wts = np.array([gw[a] * gw[c] * hx * hz for c in range(cfg.nq_u) for a in range(cfg.nq_u)])
                p4 = None
                if k is not None and act[k]:
                    p4 = np.array([psi_point(cfg, tau, e, xi) for xi in pts])
                if cfg.wall_amp != 0.0:
                    hn = _curved_wall_flux(cfg, e, pts, gw, s, sg, us, omegas, betas, f, p4, k, off, nle)
                    _add_wall_term(rhs, e, p3, pts, hn, nodes_p)
                    continue
                hn = np.zeros(len(pts))
                for u, om, beta in zip(us, omegas, betas):
                    u = np.asarray(u, dtype=np.float64)
                    om = np.asarray(om, dtype=np.float64)
                    ut = u[off + 3 * nle * k:off + 3 * nle * (k + 1)] if p4 is not None else None
                    ot = om[off + 3 * nle * k:off + 3 * nle * (k + 1)] if p4 is not None else None
                    _, val, g = _cell_grads(cfg, u, e, pts, h, p4, ut)
                    _, _, go = _cell_grads(cfg, om, e, pts, h, p4, ot)
                    div = g[:, 0, 0] + g[:, 1, 1] + g[:, 2, 2]
                    conv_y = np.einsum("qj,qj->q", g[:, 1, :], val) + val[:, 1] * div
                    curl_y = go[:, 0, 2] - go[:, 2, 0]
                    hn += beta * sg * (conv_y + cfg.nu * curl_y)
                hn = -hn + sg * f[1]
                for qi, xi in enumerate(pts):
                    vx = lagrange(nodes_p, xi[0])[0]
                    vy = lagrange(nodes_p, xi[1])[0]
                    vz = lagrange(nodes_p, xi[2])[0]
                    Np = np.einsum("m,j,i->mji", vz, vy, vx).reshape(-1)
                    rhs[e * p3:(e + 1) * p3] += wts[qi] * hn[qi] * Np
    return rhs


def _curved_wall_flux(cfg, e, pts, gw, s, sg, us, omegas, betas, f, p4, k, off, nle):
    """h_N w dA at the wall-face points pts of curved cell e: the full normal of
    the isoparametric wall, n dA = |det J| J^{-T} (sg e_y) dA_ref (Nanson), and
    div(u (x) u) = (u . grad) u + u div u, all three components."""
    from .project import basis_at, _basis_grad_at
    J = cell_jacobians(cfg, e, pts)
    Ji = np.linalg.inv(J)
    wref = np.array([gw[a] * gw[c] for c in range(cfg.nq_u) for a in range(cfg.nq_u)])
    nwda = (sg * wref * np.abs(np.linalg.det(J)))[:, None] * Ji[:, 1, :]
    V = basis_at(cfg, pts)
    G = np.einsum("qba,qad->qbd", _basis_grad_at(cfg, pts, (1.0, 1.0, 1.0)), Ji)
    n3 = (cfg.k_u + 1) ** 3
    hvec = np.zeros((len(pts), 3))
    for u, om, beta in zip(us, omegas, betas):
        u = np.asarray(u, dtype=np.float64)
        om = np.asarray(om, dtype=np.float64)
        U = u[e * 3 * n3:(e + 1) * 3 * n3].reshape(3, n3)
        W = om[e * 3 * n3:(e + 1) * 3 * n3].reshape(3, n3)
        val, g, go = V @ U.T, np.einsum("qbd,cb->qcd", G, U), np.einsum("qbd,cb->qcd", G, W)
        if p4 is not None:
            ut, ot = u[off + 3 * k:off + 3 * k + 3], om[off + 3 * k:off + 3 * k + 3]
            val += p4[:, 0:1] * ut[None, :]
            g += ut[None, :, None] * p4[:, None, 1:4]
            go += ot[None, :, None] * p4[:, None, 1:4]
        div = g[:, 0, 0] + g[:, 1, 1] + g[:, 2, 2]
        conv = np.einsum("qij,qj->qi", g, val) + val * div[:, None]
        hvec += beta * (conv + cfg.nu * _curl(go))
    return -np.einsum("qi,qi->q", hvec - np.asarray(f, dtype=np.float64)[None, :], nwda)


def _add_wall_term(rhs, e, p3, pts, hn_wda, nodes_p):
    for qi, xi in enumerate(pts):
        vx = lagrange(nodes_p, xi[0])[0]
        vy = lagrange(nodes_p, xi[1])[0]
        vz = lagrange(nodes_p, xi[2])[0]
        rhs[e * p3:(e + 1) * p3] += hn_wda[qi] * np.einsum("m,j,i->mji", vz, vy, vx).reshape(-1)


def dual_splitting_step(cfg, tau, u_n, u_nm1, dt, order=2, f=(0.0, 0.0, 0.0), dt_over_cr=None,
                        c_des=0.85, beta_des=6.0, helm_rtol=1e-11):
    """One step of the dual-splitting scheme (Sec. 4.1; the element-wise forms
    of Sec. 4.2), each step from the oracle's operators, in the paper's order:
    convective step (eq. convstepspat), pressure Poisson equation with the
    high-order Neumann data (eqs. poissonspat, ipflux, bc_d_pres; dense
    least squares, zero mean), projection (eq. projectionspat, tau_D from
    u^n), Helmholtz step (eq. helmholtzspat, nu_t from u^n).  Constant-step
    BDF/extrapolation coefficients of order 1 or 2.  Returns (u^{n+1}, p,
    u_hat, u_hathat).  With l = 1 every operator takes the degree-1
    enrichment weights (Sec. 3.1 eq. enrichment)."""
    from . import convective_residual, divdiv_tau, pressure_gradient, velocity_divergence
    from . import solve as osolve
    from .project import projection_step
    if order == 2:
        g0, al, be = 1.5, (2.0, -0.5), (2.0, -1.0)
        us = [np.asarray(u_n, dtype=np.float64), np.asarray(u_nm1, dtype=np.float64)]
    else:
        g0, al, be = 1.0, (1.0,), (1.0,)
        us = [np.asarray(u_n, dtype=np.float64)]
    dt_over_cr = dt / 0.14 if dt_over_cr is None else dt_over_cr
    n3 = (cfg.k_u + 1) ** 3
    off = cfg.ncell * 3 * n3
    psi = _psi(cfg, tau)
    # 1 convective step; M^{-1} (v, f) of a constant f is f on the polynomial unknowns
    s = sum(b * convective_residual(cfg, u, tau) for b, u in zip(be, us))
    u_hat = (sum(a * u for a, u in zip(al, us)) - dt * inverse_mass(cfg, s, psi)) / g0
    fpoly = np.zeros(cfg.n_vel)
    for c in range(3):
        for e in range(cfg.ncell):
            fpoly[(e * 3 + c) * n3:(e * 3 + c + 1) * n3] = f[c]
    u_hat += dt / g0 * fpoly
    # 2 pressure
    oms = [vorticity(cfg, u, tau) for u in us]
    rhs = -(g0 / dt) * velocity_divergence(cfg, u_hat, tau=tau) + pressure_neumann(cfg, us, oms, be, f, tau)
    p = osolve.dense_solution(cfg, rhs)
    # 3 projection
    g = pressure_gradient(cfg, p, tau=tau)
    tau_d = divdiv_tau(cfg, us[0], dt_over_cr, tau=tau)
    cells = enriched_cells(cfg)
    psi4 = psi_volume4(cfg, cells, tau=tau) if cells.size else np.zeros((0, 1, 4))
    u_hh = projection_step(cfg, u_hat, g, dt / g0, tau_d, psi4)
    # 4 Helmholtz
    u_np1, _ = helmholtz_solve(cfg, us[0], tau, g0 / dt, u_hh, rtol=helm_rtol)
    del off
    return u_np1, p, u_hat, u_hh
