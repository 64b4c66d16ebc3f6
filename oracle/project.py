"""Cell-wise L2 projection onto the refreshed enriched space (arXiv
1705.08813, Sec. 3.2, eq. l2), and the inverse of the velocity mass matrix.

TEST INFRASTRUCTURE ONLY (never used by the product).

When the wall shear stress changes, the enrichment function of every
enriched cell changes from psi_old to psi_new, and the velocity is carried
into the new space cell by cell:

    int_e v . u_new dOmega = int_e v . u_old dOmega   for every v of the new local space.

The new local space of an enriched cell is span{N_B e_c} together with
psi_new e_c while its enrichment is on, the polynomial span alone while it is
switched off (psi_new identically zero); u_old = u_bar_old + psi_old u~_old.
With the enriched cell's quadrature rule (nq_u x nq_wn x nq_u Gauss points,
weights w_q times |det J|) eq. l2 is the normal equation of the weighted
least-squares problem  min_x || W^{1/2} (Phi x - u_old) ||  with Phi the new
local basis evaluated at the points: every enriched cell forms Phi directly
from 3-D basis values and solves that problem with numpy's least-squares
routine (SVD), which gives the solution of eq. l2 without squaring the
condition number of the mass matrix Phi^T W Phi (about 5e6 when psi is close
to a polynomial on the cell).  The three velocity components decouple (the
basis is componentwise).  Cells without enrichment
keep their values, since their space does not change.

psi_old and psi_new are given as values at those quadrature points
([enriched cell][point], x fastest, then the wall-normal rule, then z), so
that tests can also feed synthetic fields.  The L2 projection and the
projection step are for flat (box) meshes; the mass matrix and its inverse
also take the curved-wall mesh (l = 0, |det J| per point).
"""
from __future__ import annotations

import numpy as np

from . import cell_map, enriched_cells, gauss, gauss_lobatto, lagrange, vertex_eta


def volume_rule(cfg):
    """Reference points (npts, 3) and weights of the enriched volume rule."""
    qu, wu = gauss(cfg.nq_u)
    qw, ww = gauss(cfg.nq_wn)
    pts, wts = [], []
    for c in range(cfg.nq_u):
        for b in range(cfg.nq_wn):
            for a in range(cfg.nq_u):
                pts.append((qu[a], qw[b], qu[c]))
                wts.append(wu[a] * ww[b] * wu[c])
    return np.array(pts), np.array(wts)


def basis_at(cfg, pts):
    """N_B at the points, B = i + n (j + n m): array (npts, n^3)."""
    n = cfg.k_u + 1
    nodes = gauss_lobatto(n)
    V = np.zeros((len(pts), n ** 3))
    for q, (x, y, z) in enumerate(pts):
        vx, vy, vz = lagrange(nodes, x)[0], lagrange(nodes, y)[0], lagrange(nodes, z)[0]
        V[q] = np.einsum("m,j,i->mji", vz, vy, vx).reshape(-1)
    return V


def project(cfg, u_old, psi_old, psi_new, return_cond=False, only=None):
    """u_new of eq. l2.  psi_old, psi_new: [nenr][npts] values at the enriched
    volume rule.  With return_cond, also the 2-norm condition number of each
    enriched cell's mass matrix.  only: enriched-cell positions to project
    (the projection is cell-local; the others keep u_old).  With l = 1 the
    old and new enrichment functions are psi N_B (Sec. 3.1 eq. enrichment)."""
    if cfg.wall_amp != 0.0:
        raise ValueError("flat meshes only")
    n3 = (cfg.k_u + 1) ** 3
    u_old = np.asarray(u_old, dtype=np.float64)
    u_new = u_old.copy()
    cells = enriched_cells(cfg)
    pts, wts = volume_rule(cfg)
    V = basis_at(cfg, pts)
    eta = vertex_eta(cfg)
    off = cfg.ncell * 3 * n3
    conds = np.zeros(len(cells))
    todo = range(len(cells)) if only is None else sorted(set(int(k) for k in only))
    nle = _nle(cfg)
    for k in todo:
        e = cells[k]
        w, Phi, uq, on = _l2_cell(cfg, k, u_old, psi_old[k], psi_new[k], V, wts, eta, cells)
        sw = np.sqrt(w)
        A = sw[:, None] * Phi
        conds[k] = np.linalg.cond(A.T @ A)
        for c in range(3):
            x = np.linalg.lstsq(A, sw * uq[c], rcond=None)[0]
            u_new[(e * 3 + c) * n3:(e * 3 + c + 1) * n3] = x[:n3]
            u_new[off + nle * (3 * k + c):off + nle * (3 * k + c + 1)] = x[n3:] if on else 0.0
    return (u_new, conds) if return_cond else u_new


def _l2_cell(cfg, k, u_old, psi_old_k, psi_new_k, V, wts, eta, cells):
    """Quadrature weights w (times |det J|), the new local basis Phi at the
    points, the old velocity uq[c] at the points and the activity of enriched
    cell k (position in enrichment order)."""
    n3 = (cfg.k_u + 1) ** 3
    hx, hz = cfg.Lx / cfg.nx, cfg.Lz / cfg.nz
    off = cfg.ncell * 3 * n3
    e = cells[k]
    ey = (e // cfg.nx) % cfg.ny
    detJ = hx * (eta[ey + 1] - eta[ey]) * hz
    w = wts * detJ
    po, pn = np.asarray(psi_old_k, dtype=float), np.asarray(psi_new_k, dtype=float)
    nle = _nle(cfg)
    Nl = _vertex_fns(volume_rule(cfg)[0]) if nle == 8 else np.ones((len(po), 1))   # N^l_B at the points
    on = bool(np.any(pn != 0.0))
    Phi = np.hstack([V, pn[:, None] * Nl]) if on else V      # new local basis at the points
    uq = []
    for c in range(3):
        ub = u_old[(e * 3 + c) * n3:(e * 3 + c + 1) * n3]
        ut = u_old[off + nle * (3 * k + c):off + nle * (3 * k + c + 1)]
        uq.append(V @ ub + po * (Nl @ ut))                   # u_old at the points
    return w, Phi, uq, on


def l2_normal_equation(cfg, k, u_old, psi_old_k, psi_new_k):
    """Eq. l2 of enriched cell k written as its normal equation A x_c = b_c per
    component c: A = Phi^T W Phi (the new local mass matrix), b_c = Phi^T W u_old,c,
    and babs_c = |Phi|^T W |u_old,c| (a bound on the rounding of b_c)."""
    cells = enriched_cells(cfg)
    pts, wts = volume_rule(cfg)
    V = basis_at(cfg, pts)
    w, Phi, uq, _ = _l2_cell(cfg, k, np.asarray(u_old, dtype=float), psi_old_k, psi_new_k, V, wts,
                             vertex_eta(cfg), cells)
    A = Phi.T @ (w[:, None] * Phi)
    b = [Phi.T @ (w * q) for q in uq]
    babs = [np.abs(Phi).T @ (w * np.abs(q)) for q in uq]
    return A, b, babs


def inverse_mass(cfg, r, psi, cells=None, return_cond=False):
    """x = M^{-1} r for the velocity mass matrix of every cell (the operator
    of the semi-discrete system M du/dt = -R(u), Sec. 4.1-4.2): per cell and
    component M_ij = (phi_i, phi_j)_e with phi the cell's local basis (N_B,
    plus psi in an enriched cell whose enrichment is on) and the cell's own
    quadrature rule (nq_u^3, or nq_u x nq_wn x nq_u in enriched cells),
    assembled directly from 3-D basis values and solved densely.  psi:
    [nenr][npts] values at the enriched volume rule (zero rows: enrichment
    switched off, its unknowns set to 0).  cells: the cells to invert (the
    operator is block diagonal; the others are left at 0).  With return_cond,
    also the 2-norm condition number of each cell's block (0 for cells not
    inverted).  On the curved-wall mesh (l = 0) |det J| enters per point.
    With degree-1 enrichment weights
    (Sec. 3.1 eq. enrichment, l = 1) the enrichment functions of a cell are
    psi N_B, N_B its eight trilinear vertex functions."""
    if cfg.wall_amp != 0.0 and _nle(cfg) != 1:
        raise ValueError("curved meshes: l = 0 only")
    n3 = (cfg.k_u + 1) ** 3
    r = np.asarray(r, dtype=np.float64)
    x = np.zeros_like(r)
    eta = vertex_eta(cfg)
    off = cfg.ncell * 3 * n3
    enr = {int(e): k for k, e in enumerate(enriched_cells(cfg))}
    pts_e, wts_e = volume_rule(cfg)
    V_e = basis_at(cfg, pts_e)
    pts_r, wts_r = volume_rule(cfg.with_(nq_wn=cfg.nq_u))
    V_r = basis_at(cfg, pts_r)
    M_reg = V_r.T @ (wts_r[:, None] * V_r)
    conds = np.zeros(cfg.ncell)
    nle = _nle(cfg)
    for e in (range(cfg.ncell) if cells is None else [int(c) for c in cells]):
        k = enr.get(e)
        M = _mass_block(cfg, e, None if k is None else psi[k], eta, M_reg, V_e, wts_e, pts_e, (pts_r, wts_r, V_r))
        conds[e] = np.linalg.cond(M)
        for c in range(3):
            rp = r[(e * 3 + c) * n3:(e * 3 + c + 1) * n3]
            if k is not None and M.shape[0] == n3 + nle:
                o = off + (3 * k + c) * nle
                sol = np.linalg.solve(M, np.concatenate([rp, r[o:o + nle]]))
                x[o:o + nle] = sol[n3:]
                x[(e * 3 + c) * n3:(e * 3 + c + 1) * n3] = sol[:n3]
            else:
                x[(e * 3 + c) * n3:(e * 3 + c + 1) * n3] = np.linalg.solve(M, rp)
    return (x, conds) if return_cond else x


def mass_apply(cfg, x, psi):
    """y = M x with the velocity mass matrix of every cell (the forward
    operator that inverse_mass inverts; same blocks, same psi convention:
    zero rows switch a cell's enrichment off, its unknowns then map to 0)."""
    if cfg.wall_amp != 0.0 and _nle(cfg) != 1:
        raise ValueError("curved meshes: l = 0 only")
    n3 = (cfg.k_u + 1) ** 3
    x = np.asarray(x, dtype=np.float64)
    y = np.zeros_like(x)
    eta = vertex_eta(cfg)
    off = cfg.ncell * 3 * n3
    enr = {int(e): k for k, e in enumerate(enriched_cells(cfg))}
    pts_e, wts_e = volume_rule(cfg)
    V_e = basis_at(cfg, pts_e)
    pts_r, wts_r = volume_rule(cfg.with_(nq_wn=cfg.nq_u))
    V_r = basis_at(cfg, pts_r)
    M_reg = V_r.T @ (wts_r[:, None] * V_r)
    nle = _nle(cfg)
    for e in range(cfg.ncell):
        k = enr.get(e)
        M = _mass_block(cfg, e, None if k is None else psi[k], eta, M_reg, V_e, wts_e, pts_e, (pts_r, wts_r, V_r))
        for c in range(3):
            xp = x[(e * 3 + c) * n3:(e * 3 + c + 1) * n3]
            if k is not None and M.shape[0] == n3 + nle:
                o = off + (3 * k + c) * nle
                v = M @ np.concatenate([xp, x[o:o + nle]])
                y[(e * 3 + c) * n3:(e * 3 + c + 1) * n3] = v[:n3]
                y[o:o + nle] = v[n3:]
            else:
                y[(e * 3 + c) * n3:(e * 3 + c + 1) * n3] = M @ xp
    return y


def _nle(cfg):
    """Enrichment functions per component and enriched cell: (l+1)^3."""
    return (getattr(cfg, "enrich_degree", 0) + 1) ** 3


def _vertex_grads(pts, h):
    """Trilinear vertex functions N_B (B = bx + 2 (by + 2 bz)) at reference
    points and their physical gradients (h: cell sizes): (npts, 8), (npts, 8, 3)."""
    pts = np.asarray(pts, dtype=np.float64)
    N = np.ones((len(pts), 8))
    dN = np.ones((len(pts), 8, 3))
    for b in range(8):
        for d in range(3):
            on = (b >> d) & 1
            f = pts[:, d] if on else 1.0 - pts[:, d]
            N[:, b] *= f
            for dd in range(3):
                dN[:, b, dd] *= ((1.0 if on else -1.0) / h[d]) if dd == d else f
    return N, dN


def _vertex_fns(pts):
    """Trilinear vertex functions N_B (B = bx + 2 (by + 2 bz)) at reference points: (npts, 8)."""
    N = np.ones((len(pts), 8))
    for B in range(8):
        for d in range(3):
            N[:, B] *= pts[:, d] if (B >> d) & 1 else 1.0 - pts[:, d]
    return N


def _curved_detj(cfg, e, pts):
    """|det J| at the reference points pts of cell e of the curved-wall mesh
    (its degree-k_u isoparametric map, Sec. 5.2 geometry)."""
    return np.abs(np.array([cell_map(cfg, e, p)[1] for p in pts]))


def _mass_block(cfg, e, psi_k, eta, M_reg, V_e, wts_e, pts_e=None, reg=None):
    """Per-component mass matrix of cell e over its local basis (N_B, plus the
    enrichment functions psi N^l_B while an enriched cell's enrichment is on),
    the cell's own rule.  On the curved-wall mesh |det J| varies over the cell
    and enters point by point (reg: points, weights and basis values of the
    regular rule, for the cells without enrichment)."""
    if cfg.wall_amp != 0.0:
        pts, wts, V = reg if psi_k is None else (pts_e, wts_e, V_e)
        w = wts * _curved_detj(cfg, e, pts)
        if psi_k is None:
            return V.T @ (w[:, None] * V)
        ps = np.asarray(psi_k, dtype=float)
        Phi = np.hstack([V, ps[:, None]]) if np.any(ps != 0.0) else V
        return Phi.T @ (w[:, None] * Phi)
    hx, hz = cfg.Lx / cfg.nx, cfg.Lz / cfg.nz
    ey = (e // cfg.nx) % cfg.ny
    detJ = hx * (eta[ey + 1] - eta[ey]) * hz
    if psi_k is None:
        return detJ * M_reg
    ps = np.asarray(psi_k, dtype=float)
    on = bool(np.any(ps != 0.0))
    if _nle(cfg) == 1:
        E = ps[:, None]
    else:
        E = ps[:, None] * _vertex_fns(volume_rule(cfg)[0] if pts_e is None else pts_e)
    Phi = np.hstack([V_e, E]) if on else V_e
    return Phi.T @ ((detJ * wts_e)[:, None] * Phi)


def mass_block(cfg, e, psi_k=None):
    """The block of cell e that inverse_mass inverts, per component: (n+1) x (n+1)
    with n = (k_u+1)^3 in an enriched cell whose enrichment is on (psi_k: psi at
    the enriched volume rule), n x n otherwise (psi_k None for a cell without
    enrichment)."""
    pts_e, wts_e = volume_rule(cfg)
    V_e = basis_at(cfg, pts_e)
    pts_r, wts_r = volume_rule(cfg.with_(nq_wn=cfg.nq_u))
    V_r = basis_at(cfg, pts_r)
    M_reg = V_r.T @ (wts_r[:, None] * V_r)
    return _mass_block(cfg, int(e), psi_k, vertex_eta(cfg), M_reg, V_e, wts_e, pts_e, (pts_r, wts_r, V_r))


def _basis_grad_at(cfg, pts, h):
    """Physical gradients of N_B at the points: array (npts, n^3, 3)."""
    n = cfg.k_u + 1
    nodes = gauss_lobatto(n)
    G = np.zeros((len(pts), n ** 3, 3))
    for q, (x, y, z) in enumerate(pts):
        (vx, dx), (vy, dy), (vz, dz) = lagrange(nodes, x), lagrange(nodes, y), lagrange(nodes, z)
        G[q, :, 0] = np.einsum("m,j,i->mji", vz, vy, dx).reshape(-1) / h[0]
        G[q, :, 1] = np.einsum("m,j,i->mji", vz, dy, vx).reshape(-1) / h[1]
        G[q, :, 2] = np.einsum("m,j,i->mji", dz, vy, vx).reshape(-1) / h[2]
    return G


def _projection_block(cfg, e, psi4_k, tau_d_e, eta, rule_e, rule_r):
    """M_e and D_e of eq. projectionspat over the local basis of cell e (the
    three components of N_B, plus the enrichment functions psi N^l_B e_c
    while the enrichment is on: psi e_c for l = 0)."""
    n3 = (cfg.k_u + 1) ** 3
    hx, hz = cfg.Lx / cfg.nx, cfg.Lz / cfg.nz
    ey = (e // cfg.nx) % cfg.ny
    h = (hx, eta[ey + 1] - eta[ey], hz)
    detJ = h[0] * h[1] * h[2]
    pts, wts, V = rule_e if psi4_k is not None else rule_r
    G = _basis_grad_at(cfg, pts, h)
    w = wts * detJ
    on = psi4_k is not None and bool(np.any(psi4_k[:, 0] != 0.0))
    nle = _nle(cfg)
    nb = 3 * n3 + (3 * nle if on else 0)
    if on:
        # enrichment functions and their gradients: psi N_B, N_B grad psi + psi grad N_B
        N, dN = _vertex_grads(pts, h) if nle == 8 else (np.ones((len(pts), 1)), np.zeros((len(pts), 1, 3)))
        phi = psi4_k[:, 0:1] * N
        gphi = N[:, :, None] * psi4_k[:, None, 1:4] + psi4_k[:, 0, None, None] * dN
    # values (npts, 3, nb) and divergences (npts, nb) of the local basis
    val = np.zeros((len(pts), 3, nb))
    div = np.zeros((len(pts), nb))
    for c in range(3):
        val[:, c, c * n3:(c + 1) * n3] = V
        div[:, c * n3:(c + 1) * n3] = G[:, :, c]
        if on:
            val[:, c, 3 * n3 + c * nle:3 * n3 + (c + 1) * nle] = phi
            div[:, 3 * n3 + c * nle:3 * n3 + (c + 1) * nle] = gphi[:, :, c]
    M = np.einsum("q,qci,qcj->ij", w, val, val)
    D = tau_d_e * np.einsum("q,qi,qj->ij", w, div, div)
    return M, D, on


def projection_block(cfg, e, tau_d_e, psi4_k=None):
    """(M_e, D_e) of the projection step for cell e: 3 n (+3 (l+1)^3 while an
    enriched cell's enrichment is on) square, unknowns ordered as in the
    velocity layout (components of N_B, then the enrichment coefficients
    [c][B]).  psi4_k: psi and grad psi at the enriched volume rule, None for a
    cell without enrichment."""
    pts_e, wts_e = volume_rule(cfg)
    pts_r, wts_r = volume_rule(cfg.with_(nq_wn=cfg.nq_u))
    M, D, _ = _projection_block(cfg, int(e), psi4_k, tau_d_e, vertex_eta(cfg),
                                (pts_e, wts_e, basis_at(cfg, pts_e)), (pts_r, wts_r, basis_at(cfg, pts_r)))
    return M, D


def projection_step(cfg, u_hat, g, scale, tau_d, psi4, cells=None):
    """The element-wise projection step of the dual-splitting scheme (Sec.
    4.2, eq. projectionspat):  M_e(v, x) + D_e(v, x) = M_e(v, u_hat) - scale P_e(v, p)
    for every velocity test function v of every cell, with g = P p given
    (velocity layout) and D_e the div-div penalty (div v, tau_D,e div x)_e.
    Per cell the matrix M_e + D_e over the cell's local basis (3 components
    of N_B, plus psi e_c while the enrichment is on; the cell's velocity
    rule) is assembled from 3-D basis values and gradients and the system is
    solved densely.  psi4: [nenr][npts][4] psi and grad psi at the enriched
    volume rule.  cells: optional subset of cells to solve (others stay 0).
    With l = 1 the enrichment functions are psi N_B e_c (Sec. 3.1 eq.
    enrichment).  Flat (box) meshes only."""
    if cfg.wall_amp != 0.0:
        raise ValueError("flat meshes only")
    n3 = (cfg.k_u + 1) ** 3
    u_hat = np.asarray(u_hat, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    x = np.zeros_like(u_hat)
    eta = vertex_eta(cfg)
    off = cfg.ncell * 3 * n3
    enr = {int(e): k for k, e in enumerate(enriched_cells(cfg))}
    pts_e, wts_e = volume_rule(cfg)
    pts_r, wts_r = volume_rule(cfg.with_(nq_wn=cfg.nq_u))
    V_e, V_r = basis_at(cfg, pts_e), basis_at(cfg, pts_r)
    ne = 3 * _nle(cfg)
    for e in (range(cfg.ncell) if cells is None else (int(c) for c in cells)):
        k = enr.get(e)
        M, D, on = _projection_block(cfg, e, None if k is None else psi4[k], tau_d[e], eta,
                                     (pts_e, wts_e, V_e), (pts_r, wts_r, V_r))
        # right-hand side: M u_hat - scale g
        coef = np.concatenate([u_hat[e * 3 * n3:(e + 1) * 3 * n3]] + ([u_hat[off + ne * k: off + ne * (k + 1)]] if on else []))
        rhs = M @ coef - scale * np.concatenate([g[e * 3 * n3:(e + 1) * 3 * n3]] +
                                                ([g[off + ne * k: off + ne * (k + 1)]] if on else []))
        sol = np.linalg.solve(M + D, rhs)
        x[e * 3 * n3:(e + 1) * 3 * n3] = sol[:3 * n3]
        if k is not None:
            x[off + ne * k: off + ne * (k + 1)] = sol[3 * n3:] if on else 0.0
    return x
