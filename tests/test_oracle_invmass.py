"""Pins of the oracle's inverse velocity mass matrix (the M of M du/dt = -R(u)).

The right-hand side r = M x is formed independently of the oracle: for x the
nodal values of a polynomial p in Q_k plus an enrichment coefficient c with a
synthetic enrichment function q (a polynomial of degree k+1 in the
wall-normal coordinate, outside Q_k), every entry r_B = (N_B, p + c q)_e and
r_e = (q, p + c q)_e is an integral of a polynomial that both the cell's rule
and a 12-point numpy Gauss rule integrate exactly, so it is computed with the
latter and a Vandermonde-inverse basis; M^{-1} r must return x.
"""
import numpy as np
import pytest

from oracle import dense
from oracle import project as OP
import oracle as O
from paper_1705_08813_amd.inputs import MeshConfig


def _cell_moments(cfg, e, f_ref):
    """(N_B, f)_e and (q, f)_e for f given as a function of reference coordinates,
    with the 12-point Gauss rule and the Vandermonde basis."""
    n = cfg.k_u + 1
    g, w = dense.gauss01(12)
    Nb, _ = dense.basis1d(dense.lobatto01(n), g)            # (12, n)
    eta = O.vertex_eta(cfg)
    ey = (e // cfg.nx) % cfg.ny
    detJ = cfg.Lx / cfg.nx * (eta[ey + 1] - eta[ey]) * cfg.Lz / cfg.nz
    Z, Y, X = np.meshgrid(g, g, g, indexing="ij")
    W = (w[:, None, None] * w[None, :, None] * w[None, None, :]) * detJ
    F = f_ref(X, Y, Z) * W
    # r[m, j, i] = sum_{z,y,x} Nz[z,m] Ny[y,j] Nx[x,i] F[z,y,x]
    r = np.einsum("zm,yj,xi,zyx->mji", Nb, Nb, Nb, F).reshape(-1)
    return r, W


P_COEF = np.random.default_rng(3).uniform(-1, 1, 5)


def _p(k):
    a = P_COEF
    return lambda X, Y, Z: a[0] + a[1] * X ** k * Y + a[2] * Y ** k * Z ** (k - 1) + a[3] * X * Z ** k + a[4] * (X * Y * Z) ** k


def _q(k):
    return lambda X, Y, Z: Y ** (k + 1) + 0.3 * X * Y ** (k + 1) - 0.2 * Z


@pytest.mark.parametrize("cfg", [MeshConfig(nx=2, ny=3, nz=2, gamma=1.0, k_u=3, nq_u=5, nq_wn=8),
                                 MeshConfig(nx=2, ny=3, nz=1, gamma=0.6, k_u=4, nq_u=7, nq_wn=8),
                                 MeshConfig(nx=1, ny=3, nz=2, gamma=1.4, k_u=2, nq_u=4, nq_wn=8, enrich_upper=0)])
def test_inverse_mass_recovers_polynomials_and_enrichment(cfg):
    k = cfg.k_u
    n3 = (k + 1) ** 3
    p, q = _p(k), _q(k)
    cells = O.enriched_cells(cfg)
    pts, _ = OP.volume_rule(cfg)
    psi = np.array([q(pts[:, 0], pts[:, 1], pts[:, 2]) for _ in cells])
    c = np.array([0.7, -1.3, 0.4])
    r = np.zeros(cfg.n_vel)
    off = cfg.ncell * 3 * n3
    enr = {int(e): kk for kk, e in enumerate(cells)}
    g = dense.lobatto01(k + 1)
    Zn, Yn, Xn = np.meshgrid(g, g, g, indexing="ij")
    pn = p(Xn, Yn, Zn).reshape(-1)
    x_expect = np.zeros(cfg.n_vel)
    for e in range(cfg.ncell):
        kk = enr.get(e)
        for comp in range(3):
            s = 1.0 + comp
            if kk is None:
                rb, _ = _cell_moments(cfg, e, lambda X, Y, Z: s * p(X, Y, Z))
            else:
                f = lambda X, Y, Z: s * p(X, Y, Z) + c[comp] * q(X, Y, Z)
                rb, W = _cell_moments(cfg, e, f)
                g12 = dense.gauss01(12)[0]
                Z, Y, X = np.meshgrid(g12, g12, g12, indexing="ij")
                r[off + 3 * kk + comp] = np.sum(W * q(X, Y, Z) * f(X, Y, Z))
                x_expect[off + 3 * kk + comp] = c[comp]
            r[(e * 3 + comp) * n3:(e * 3 + comp + 1) * n3] = rb
            x_expect[(e * 3 + comp) * n3:(e * 3 + comp + 1) * n3] = s * pn
    x = OP.inverse_mass(cfg, r, psi)
    np.testing.assert_allclose(x, x_expect, rtol=0, atol=1e-9 * np.abs(x_expect).max())


def test_switched_off_cell_inverts_the_polynomial_block():
    cfg = MeshConfig(nx=2, ny=3, nz=2, gamma=1.0, k_u=3, nq_u=5, nq_wn=8)
    k = cfg.k_u
    n3 = (k + 1) ** 3
    p = _p(k)
    cells = O.enriched_cells(cfg)
    psi = np.zeros((cells.size, cfg.nq_u * cfg.nq_wn * cfg.nq_u))
    r = np.zeros(cfg.n_vel)
    off = cfg.ncell * 3 * n3
    r[off:] = 5.0                       # ignored: the enrichment is off
    g = dense.lobatto01(k + 1)
    Zn, Yn, Xn = np.meshgrid(g, g, g, indexing="ij")
    pn = p(Xn, Yn, Zn).reshape(-1)
    for e in cells:
        rb, _ = _cell_moments(cfg, e, p)
        r[(e * 3) * n3:(e * 3 + 1) * n3] = rb
    x = OP.inverse_mass(cfg, r, psi)
    assert np.all(x[off:] == 0.0)
    for e in cells:
        np.testing.assert_allclose(x[(e * 3) * n3:(e * 3 + 1) * n3], pn, rtol=0, atol=1e-10)
