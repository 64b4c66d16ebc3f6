"""Face-by-face dense assembly of the linear operators on small box meshes.

TEST INFRASTRUCTURE ONLY (pins the C oracle; never used by the product).

This is a second, independent formulation of the two linear bilinear forms of
Sec. 4.2 of arXiv 1705.08813:
  * the SIP pressure Laplace form (eq. ipflux, homogeneous Neumann walls),
  * the symmetric/nonsymmetric interior-penalty viscous form (last row of
    eq. viscous_multiscale with the adjoint sign theta, nu_t = 0, mirror
    values on no-slip walls and the x10 wall penalty).
Unlike the C oracle (element by element, each cell evaluating both traces),
it visits every face once and writes the symmetric face form
  -[q]{{d_n p}} - {{d_n q}}[p] + tau [q][p]
into the rows and columns of both cells.  The 1-D bases are built from the
inverse Vandermonde matrix (not the Lagrange product formula) and the rules
come from numpy's Gauss-Legendre routine.  Box meshes only (affine cells).
"""
from __future__ import annotations

import numpy as np


def gauss01(n):
    t, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (t + 1.0), 0.5 * w


def lobatto01(n):
    inner = np.polynomial.legendre.Legendre.basis(n - 1).deriv().roots()
    t = np.concatenate([[-1.0], np.sort(np.real(inner)), [1.0]])
    return 0.5 * (t + 1.0)


def basis1d(nodes, t):
    """Values and derivatives of the Lagrange basis through `nodes` at points t
    via monomial coefficients C = V^{-1}."""
    nodes = np.asarray(nodes, dtype=float)
    n = len(nodes)
    C = np.linalg.inv(np.vander(nodes, n, increasing=True))  # N_i(t) = sum_p C[p,i] t^p
    t = np.atleast_1d(np.asarray(t, dtype=float))
    T = np.vander(t, n, increasing=True)
    dT = np.zeros_like(T)
    for p in range(1, n):
        dT[:, p] = p * t ** (p - 1)
    return T @ C, dT @ C


def _mesh(cfg):
    nx, ny, nz = cfg.nx, cfg.ny, cfg.nz
    if cfg.gamma > 0:
        s = np.arange(ny + 1) / ny
        yv = np.tanh(cfg.gamma * (2 * s - 1)) / np.tanh(cfg.gamma)
    else:
        yv = np.linspace(-1.0, 1.0, ny + 1)
    hx = cfg.Lx / nx
    hz = cfg.Lz / nz
    return hx, np.diff(yv), hz


def _cell(cfg, ex, ey, ez):
    return ex + cfg.nx * (ey + cfg.ny * ez)


class _Tab:
    """3-D tensor tables of a degree (n-1) nodal basis at a tensor point set."""

    def __init__(self, nodes, pts):
        # pts: list of three 1-D arrays of reference coordinates
        self.v = []
        self.d = []
        for a in range(3):
            v, d = basis1d(nodes, pts[a])
            self.v.append(v)
            self.d.append(d)

    def values(self):
        vx, vy, vz = self.v
        return np.einsum("ai,bj,cm->cbamji", vx, vy, vz).reshape(
            vz.shape[0] * vy.shape[0] * vx.shape[0], -1)

    def grads(self, h):
        vx, vy, vz = self.v
        dx, dy, dz = self.d
        gx = np.einsum("ai,bj,cm->cbamji", dx, vy, vz) / h[0]
        gy = np.einsum("ai,bj,cm->cbamji", vx, dy, vz) / h[1]
        gz = np.einsum("ai,bj,cm->cbamji", vx, vy, dz) / h[2]
        nq = vz.shape[0] * vy.shape[0] * vx.shape[0]
        return np.stack([g.reshape(nq, -1) for g in (gx, gy, gz)], axis=-1)  # [q, B, d]


def _add_pair(A, blk, e, f, m):
    """Scatter a 2x2 block face matrix into the rows/columns of cells e and f
    (block by block, so that e == f, a cell that is its own periodic
    neighbour, accumulates correctly)."""
    cells = (e, f)
    for a in range(2):
        for b in range(2):
            A[cells[a] * m:(cells[a] + 1) * m, cells[b] * m:(cells[b] + 1) * m] += blk[a * m:(a + 1) * m, b * m:(b + 1) * m]


def _face_pts(d, s, q):
    pts = [q, q, q]
    pts[d] = np.array([float(s)])
    return pts


def poisson_matrix(cfg):
    """Dense SIP Laplace matrix A = -L (rows: test q, columns: trial p)."""
    n = cfg.k_p + 1
    np3 = n ** 3
    nodes = lobatto01(n)
    q, w = gauss01(cfg.nq_p)
    hx, hy, hz = _mesh(cfg)
    ncell = cfg.nx * cfg.ny * cfg.nz
    A = np.zeros((ncell * np3, ncell * np3))
    W3 = np.einsum("c,b,a->cba", w, w, w).ravel()
    W2 = np.einsum("b,a->ba", w, w).ravel()
    tab = _Tab(nodes, [q, q, q])
    for ez in range(cfg.nz):
        for ey in range(cfg.ny):
            for ex in range(cfg.nx):
                e = _cell(cfg, ex, ey, ez)
                h = (hx, hy[ey], hz)
                G = tab.grads(h)
                sl = slice(e * np3, (e + 1) * np3)
                A[sl, sl] += np.einsum("q,qid,qjd->ij", W3 * h[0] * h[1] * h[2], G, G)
    # each face once: the face at xi_d = 1 of every cell, neighbour across it
    for ez in range(cfg.nz):
        for ey in range(cfg.ny):
            for ex in range(cfg.nx):
                e = _cell(cfg, ex, ey, ez)
                idx = [ex, ey, ez]
                for d in range(3):
                    nmax = (cfg.nx, cfg.ny, cfg.nz)[d]
                    j = idx[d] + 1
                    if j == nmax:
                        if d == 1 and not cfg.fully_periodic:
                            continue  # upper wall: Neumann, no terms
                        j = 0
                    nidx = list(idx)
                    nidx[d] = j
                    f = _cell(cfg, *nidx)
                    he = (hx, hy[ey], hz)
                    hf = (hx, hy[nidx[1]], hz)
                    t1, t2 = [a for a in range(3) if a != d]
                    area = he[t1] * he[t2]
                    tau = cfg.ip_factor_p * n * n * max(1.0 / he[d], 1.0 / hf[d])
                    tm = _Tab(nodes, _face_pts(d, 1, q))
                    tp = _Tab(nodes, _face_pts(d, 0, q))
                    vm = tm.values()
                    vp = tp.values()
                    dm = tm.grads(he)[:, :, d]  # normal n = +e_d
                    dp = tp.grads(hf)[:, :, d]
                    wf = W2 * area
                    # jump [p] = p- - p+, average {{d_n p}}
                    jump = np.concatenate([vm, -vp], axis=1)
                    avg = 0.5 * np.concatenate([dm, dp], axis=1)
                    blk = (-np.einsum("q,qi,qj->ij", wf, jump, avg) - np.einsum("q,qi,qj->ij", wf, avg, jump)
                           + tau * np.einsum("q,qi,qj->ij", wf, jump, jump))
                    _add_pair(A, blk, e, f, np3)
    return A


def viscous_matrix(cfg):
    """Dense interior-penalty viscous matrix on the polynomial space (no
    enrichment): a(phi,u) = (2 nu eps(phi), eps(u)) - [phi].{{2nu eps(u)}}n
    - theta {{2nu eps(phi)}}n.[u] + tau nu [phi].[u], mirror data on walls."""
    n = cfg.k_u + 1
    np3 = n ** 3
    nd = 3 * np3
    nodes = lobatto01(n)
    q, w = gauss01(cfg.nq_u)
    hx, hy, hz = _mesh(cfg)
    nu, theta = cfg.nu, cfg.theta
    ncell = cfg.nx * cfg.ny * cfg.nz
    A = np.zeros((ncell * nd, ncell * nd))
    W3 = np.einsum("c,b,a->cba", w, w, w).ravel()
    W2 = np.einsum("b,a->ba", w, w).ravel()
    tab = _Tab(nodes, [q, q, q])

    def vec_tables(V, G):
        """Per point: value (3, 3*np3) and strain eps (3,3, 3*np3) of the vector
        basis N_B e_c (columns ordered [c][B])."""
        nq = V.shape[0]
        val = np.zeros((nq, 3, nd))
        eps = np.zeros((nq, 3, 3, nd))
        for c in range(3):
            val[:, c, c * np3:(c + 1) * np3] = V
            for d in range(3):
                # grad(N e_c)[c][d] = dN/dx_d
                eps[:, c, d, c * np3:(c + 1) * np3] += 0.5 * G[:, :, d]
                eps[:, d, c, c * np3:(c + 1) * np3] += 0.5 * G[:, :, d]
        return val, eps

    for ez in range(cfg.nz):
        for ey in range(cfg.ny):
            for ex in range(cfg.nx):
                e = _cell(cfg, ex, ey, ez)
                h = (hx, hy[ey], hz)
                _, eps = vec_tables(tab.values(), tab.grads(h))
                sl = slice(e * nd, (e + 1) * nd)
                A[sl, sl] += 2 * nu * np.einsum("q,qcdi,qcdj->ij", W3 * h[0] * h[1] * h[2], eps, eps)

    for ez in range(cfg.nz):
        for ey in range(cfg.ny):
            for ex in range(cfg.nx):
                e = _cell(cfg, ex, ey, ez)
                idx = [ex, ey, ez]
                he = (hx, hy[ey], hz)
                for d in range(3):
                    t1, t2 = [a for a in range(3) if a != d]
                    area = he[t1] * he[t2]
                    wf = W2 * area
                    nvec = np.zeros(3)
                    nvec[d] = 1.0
                    nmax = (cfg.nx, cfg.ny, cfg.nz)[d]
                    # lower wall face (xi_y = 0 of the first layer), outward normal -e_y
                    if d == 1 and ey == 0 and not cfg.fully_periodic:
                        tw = _Tab(nodes, _face_pts(1, 0, q))
                        val, eps = vec_tables(tw.values(), tw.grads(he))
                        nw = -nvec
                        tn = np.einsum("qcdi,d->qci", eps, nw)  # eps(phi) n
                        tau = cfg.wall_ip_mult * cfg.ip_factor_u * n * n / he[1]
                        blk = (-2 * nu * np.einsum("q,qci,qcj->ij", wf, val, tn)
                               - theta * 2 * nu * np.einsum("q,qci,qcj->ij", wf, tn, val)
                               + 2 * tau * nu * np.einsum("q,qci,qcj->ij", wf, val, val))
                        sl = slice(e * nd, (e + 1) * nd)
                        A[sl, sl] += blk
                    j = idx[d] + 1
                    if j == nmax:
                        if d == 1 and not cfg.fully_periodic:
                            tw = _Tab(nodes, _face_pts(1, 1, q))
                            val, eps = vec_tables(tw.values(), tw.grads(he))
                            tn = np.einsum("qcdi,d->qci", eps, nvec)
                            tau = cfg.wall_ip_mult * cfg.ip_factor_u * n * n / he[1]
                            blk = (-2 * nu * np.einsum("q,qci,qcj->ij", wf, val, tn)
                                   - theta * 2 * nu * np.einsum("q,qci,qcj->ij", wf, tn, val)
                                   + 2 * tau * nu * np.einsum("q,qci,qcj->ij", wf, val, val))
                            sl = slice(e * nd, (e + 1) * nd)
                            A[sl, sl] += blk
                            continue
                        j = 0
                    nidx = list(idx)
                    nidx[d] = j
                    f = _cell(cfg, *nidx)
                    hf = (hx, hy[nidx[1]], hz)
                    tm = _Tab(nodes, _face_pts(d, 1, q))
                    tp = _Tab(nodes, _face_pts(d, 0, q))
                    vm, em = vec_tables(tm.values(), tm.grads(he))
                    vp, ep = vec_tables(tp.values(), tp.grads(hf))
                    jump = np.concatenate([vm, -vp], axis=2)                      # [q, c, 2nd]
                    avg = 0.5 * np.concatenate([np.einsum("qcdi,d->qci", em, nvec),
                                                np.einsum("qcdi,d->qci", ep, nvec)], axis=2)  # {{eps}} n
                    tau = cfg.ip_factor_u * n * n * max(1.0 / he[d], 1.0 / hf[d])
                    blk = (-2 * nu * np.einsum("q,qci,qcj->ij", wf, jump, avg)
                           - theta * 2 * nu * np.einsum("q,qci,qcj->ij", wf, avg, jump)
                           + tau * nu * np.einsum("q,qci,qcj->ij", wf, jump, jump))
                    _add_pair(A, blk, e, f, nd)
    return A
