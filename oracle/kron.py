"""Kronecker-sum evaluation of the SIP Poisson operator on box meshes.

TEST INFRASTRUCTURE ONLY (pins the C oracle; never used by the product).

On a tensor-product box mesh with affine cells, the SIP Laplace form of
Sec. 4.2 (eq. ipflux) with tau_F = c (k+1)^2 max(1/h-, 1/h+) separates
exactly:  A = A_x (x) M_y (x) M_z + M_x (x) A_y (x) M_z + M_x (x) M_y (x) A_z,
where A_d is the 1-D SIP matrix of direction d (periodic in x and z,
homogeneous Neumann ends in y) and M_d the 1-D DG mass matrix.  This module
builds those 1-D matrices from numpy's Gauss rule and a Vandermonde-based
nodal basis and applies the sum by tensor contractions: a different method
from the oracle's 3-D point-by-point quadrature.
"""
from __future__ import annotations

import numpy as np

from .dense import basis1d, gauss01, lobatto01


def sip_1d(h, n, nq, periodic, ip=1.0):
    """1-D SIP stiffness (with face terms) and mass matrices on cells of sizes h."""
    ne = len(h)
    nodes = lobatto01(n)
    q, w = gauss01(nq)
    V, D = basis1d(nodes, q)
    v0, d0 = basis1d(nodes, 0.0)
    v1, d1 = basis1d(nodes, 1.0)
    v0, d0, v1, d1 = v0[0], d0[0], v1[0], d1[0]
    N = ne * n
    A = np.zeros((N, N))
    M = np.zeros((N, N))
    for e in range(ne):
        sl = slice(e * n, (e + 1) * n)
        A[sl, sl] += (D.T * w) @ D / h[e]
        M[sl, sl] += (V.T * w) @ V * h[e]
    nfaces = ne if periodic else ne - 1
    for f in range(nfaces):
        a, b = f, (f + 1) % ne            # face between cell a (left) and b (right), n = +1
        jump = np.concatenate([v1, -v0])   # [q] = q_a(1) - q_b(0)
        avg = 0.5 * np.concatenate([d1 / h[a], d0 / h[b]])
        tau = ip * n * n * max(1.0 / h[a], 1.0 / h[b])
        blk = -np.outer(jump, avg) - np.outer(avg, jump) + tau * np.outer(jump, jump)
        cells = (a, b)
        for i in range(2):
            for j in range(2):
                A[cells[i] * n:(cells[i] + 1) * n, cells[j] * n:(cells[j] + 1) * n] += blk[i * n:(i + 1) * n, j * n:(j + 1) * n]
    return A, M


def poisson_apply(cfg, p):
    """y = A p for the [cell][node] layout (cell = ex + nx(ey + ny ez),
    node = i + n(j + n m))."""
    n = cfg.k_p + 1
    nx, ny, nz = cfg.nx, cfg.ny, cfg.nz
    if cfg.gamma > 0:
        s = np.arange(ny + 1) / ny
        yv = np.tanh(cfg.gamma * (2 * s - 1)) / np.tanh(cfg.gamma)
    else:
        yv = np.linspace(-1.0, 1.0, ny + 1)
    Ax, Mx = sip_1d(np.full(nx, cfg.Lx / nx), n, cfg.nq_p, True, cfg.ip_factor_p)
    Ay, My = sip_1d(np.diff(yv), n, cfg.nq_p, bool(cfg.fully_periodic), cfg.ip_factor_p)
    Az, Mz = sip_1d(np.full(nz, cfg.Lz / nz), n, cfg.nq_p, True, cfg.ip_factor_p)
    # [ez, ey, ex, m, j, i] -> global tensor P[Z, Y, X]
    T = np.asarray(p, dtype=float).reshape(nz, ny, nx, n, n, n).transpose(0, 3, 1, 4, 2, 5)
    P = T.reshape(nz * n, ny * n, nx * n)

    def app(Z, Y, X, U):
        return np.einsum("ZK,YJ,XI,KJI->ZYX", Z, Y, X, U, optimize=True)

    Yt = app(Mz, My, Ax, P) + app(Mz, Ay, Mx, P) + app(Az, My, Mx, P)
    return Yt.reshape(nz, n, ny, n, nx, n).transpose(0, 2, 4, 1, 3, 5).reshape(-1)
