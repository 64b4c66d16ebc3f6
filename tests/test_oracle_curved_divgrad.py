"""Pins of the oracle's pressure gradient term P and velocity divergence term
C (Sec. 4.2) on the curved-wall mesh (lower wall y_w = -1 + a cos(2 pi x /
Lx), each column stretched linearly up to y = +1, isoparametric cells of
degree k_u).

  g(v) = -(div v, p)_e + (v . n, {{p}}),   c(q) = -(grad q, u)_e + (q, {{u}} . n),

with interior values on the no-slip walls.  On the mapped cells the
integrands of both terms are polynomials in the reference coordinates times
the cofactor matrix of the map (Piola), so the rules used here integrate them
exactly and the identities below hold to rounding:

  - P 1 = 0: a constant pressure exerts no net force on any test function;
  - C U = 0 for a constant velocity field U;
  - u^T P p + p^T C u = 0 when p vanishes in the wall cells (the cell-wise
    integration by parts; the interior faces cancel with central averages);
  - C applied to the field (0, y, 0), y the mapped coordinate (which the
    velocity space holds exactly), gives int_e N^p_B dV, here computed from
    the map's definition in numpy;
  - with vanishing tau_w, psi = y+ is trilinear in the reference coordinates
    and so lies in the velocity space: the enrichment rows of P are the
    polynomial rows weighted by psi at the nodes, and C of an enriched field
    equals C of the polynomial field it equals.
A wrong sign or scale of the curved normal, a transposed inverse Jacobian, a
missing |det J| or a one-sided average on interior faces fails one of them.
"""
import math

import numpy as np
import pytest

import oracle as O
from paper_1705_08813_amd.inputs import MeshConfig

CURVED = {
    "k3": MeshConfig(nx=4, ny=3, nz=2, wall_amp=0.3, k_u=3, nq_u=5, k_p=2, nq_p=3, enrich_lower=0, enrich_upper=0),
    "k5": MeshConfig(nx=3, ny=3, nz=2, wall_amp=0.3, gamma=1.2, k_u=5, nq_u=8, k_p=4, nq_p=5, enrich_lower=0,
                     enrich_upper=0),
}


def _const_velocity(cfg, U):
    n3 = (cfg.k_u + 1) ** 3
    u = np.zeros(cfg.n_vel)
    blk = u[:cfg.ncell * 3 * n3].reshape(cfg.ncell, 3, n3)
    for c in range(3):
        blk[:, c] = U[c]
    return u


@pytest.mark.parametrize("name", list(CURVED))
def test_constant_pressure_and_constant_velocity(name):
    cfg = CURVED[name]
    rng = np.random.default_rng(3)
    scale_p = np.abs(O.pressure_gradient(cfg, rng.uniform(-1, 1, cfg.n_p))).max()
    g1 = O.pressure_gradient(cfg, np.ones(cfg.n_p))
    assert np.abs(g1).max() <= 1e-13 * scale_p
    U = (0.3, -0.7, 1.1)
    scale_u = np.abs(O.velocity_divergence(cfg, rng.uniform(-1, 1, cfg.n_vel))).max()
    cu = O.velocity_divergence(cfg, _const_velocity(cfg, U))
    assert np.abs(cu).max() <= 1e-13 * scale_u


@pytest.mark.parametrize("name", list(CURVED))
def test_gradient_and_divergence_are_adjoint_away_from_walls(name):
    cfg = CURVED[name]
    rng = np.random.default_rng(4)
    npp3 = (cfg.k_p + 1) ** 3
    for _ in range(3):
        u = rng.uniform(-1, 1, cfg.n_vel)
        p = rng.uniform(-1, 1, cfg.n_p).reshape(cfg.nz, cfg.ny, cfg.nx, npp3)
        p[:, 0] = 0.0
        p[:, cfg.ny - 1] = 0.0
        p = p.ravel()
        gp, cu = O.pressure_gradient(cfg, p), O.velocity_divergence(cfg, u)
        a, b = u @ gp, p @ cu
        assert abs(a + b) <= 1e-12 * (np.abs(u) @ np.abs(gp) + np.abs(p) @ np.abs(cu))
        assert abs(a) > 1e-3 * np.abs(u) @ np.abs(gp)   # not trivially zero
    # and with p nonzero in the wall cells the identity breaks (the wall term)
    p = rng.uniform(-1, 1, cfg.n_p)
    u = rng.uniform(-1, 1, cfg.n_vel)
    gp, cu = O.pressure_gradient(cfg, p), O.velocity_divergence(cfg, u)
    assert abs(u @ gp + p @ cu) > 1e-6 * (np.abs(u) @ np.abs(gp))


def _gl_nodes(n):
    """Gauss-Lobatto nodes on [0, 1] from numpy's Legendre polynomials."""
    inner = np.sort(np.real(np.polynomial.legendre.Legendre.basis(n - 1).deriv().roots())) if n > 2 else []
    return 0.5 * (np.concatenate([[-1.0], inner, [1.0]]) + 1.0)


def _lagrange(nodes, t):
    """Lagrange basis through nodes at the points t: values and derivatives [t][i]."""
    n = len(nodes)
    v = np.ones((len(t), n))
    d = np.zeros((len(t), n))
    for i in range(n):
        for j in range(n):
            if j != i:
                v[:, i] *= (t - nodes[j]) / (nodes[i] - nodes[j])
        for m in range(n):
            if m == i:
                continue
            term = np.full(len(t), 1.0 / (nodes[i] - nodes[m]))
            for j in range(n):
                if j != i and j != m:
                    term *= (t - nodes[j]) / (nodes[i] - nodes[j])
            d[:, i] += term
    return v, d


def _curved_y(cfg, x, eta):
    """The mapped channel: y_w(x) + (eta + 1)/2 (1 - y_w(x))."""
    yw = -1.0 + cfg.wall_amp * np.cos(2.0 * math.pi * x / cfg.Lx)
    return yw + 0.5 * (eta + 1.0) * (1.0 - yw)


@pytest.mark.parametrize("name", list(CURVED))
def test_divergence_of_the_mapped_coordinate(name):
    cfg = CURVED[name]
    n, npp = cfg.k_u + 1, cfg.k_p + 1
    n3 = n ** 3
    gl, glp = _gl_nodes(n), _gl_nodes(npp)
    assert np.abs(gl - O.gauss_lobatto(n)).max() < 1e-14
    eta = O.vertex_eta(cfg)
    hx, hz = cfg.Lx / cfg.nx, cfg.Lz / cfg.nz
    u = np.zeros(cfg.n_vel)
    blk = u.reshape(cfg.ncell, 3, n3)
    Y = {}
    for e in range(cfg.ncell):
        ex, ey = e % cfg.nx, (e // cfg.nx) % cfg.ny
        X, E = np.meshgrid(ex * hx + hx * gl, eta[ey] + (eta[ey + 1] - eta[ey]) * gl, indexing="ij")  # [i][j]
        Y[e] = _curved_y(cfg, X, E)
        blk[e, 1] = np.broadcast_to(Y[e].T[None], (n, n, n)).ravel()   # [m][j][i]
    cu = O.velocity_divergence(cfg, u)
    # int_e N^p_B dV with dV = hx hz dy/dxi_y dxi, on a Gauss rule exact for these polynomials
    gq, wq = np.polynomial.legendre.leggauss(2 * n + npp)
    gq, wq = 0.5 * (gq + 1.0), 0.5 * wq
    vx, dx = _lagrange(gl, gq)              # [q][i]
    px, _ = _lagrange(glp, gq)
    for e in range(cfg.ncell):
        dydy = np.einsum("ai,bj,ij->ab", vx, dx, Y[e])          # [qx][qy]
        jac = hx * hz * dydy
        ref = np.einsum("a,b,c,ab,ai,bj,ck->kji", wq, wq, wq, jac, px, px, px).ravel()
        got = cu[e * npp ** 3:(e + 1) * npp ** 3]
        assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max(), e


def test_enrichment_rows_with_linear_psi():
    cfg = MeshConfig(nx=4, ny=3, nz=2, wall_amp=0.3, k_u=3, nq_u=5, nq_wn=8, k_p=2, nq_p=3)
    n = cfg.k_u + 1
    n3 = n ** 3
    gl = O.gauss_lobatto(n)
    tau = np.full(cfg.n_tau, 1e-14)
    s = math.sqrt(1e-14) / cfg.nu
    cells = O.enriched_cells(cfg)
    rng = np.random.default_rng(5)
    p = rng.uniform(-1, 1, cfg.n_p)
    g = O.pressure_gradient(cfg, p, tau=tau)
    ubar = rng.uniform(-1, 1, cfg.ncell * 3 * n3)
    ut = rng.uniform(-1, 1, 3 * len(cells)) / s
    up = ubar.copy().reshape(cfg.ncell, 3, n3)
    off = cfg.ncell * 3 * n3
    worst = 0.0
    for k, e in enumerate(cells):
        ps = np.array([O.psi_point(cfg, tau, int(e), (gl[B % n], gl[(B // n) % n], gl[B // (n * n)]))[0]
                       for B in range(n3)])
        assert 1e-8 < np.abs(ps).max() < 1e-4          # psi = y+ here
        for c in range(3):
            rows = g[(e * 3 + c) * n3:(e * 3 + c + 1) * n3]
            ref = ps @ rows
            worst = max(worst, abs(g[off + 3 * k + c] - ref) / (np.abs(ps) @ np.abs(rows)))
            up[e, c] += ut[3 * k + c] * ps
    assert worst <= 1e-12
    c_enr = O.velocity_divergence(cfg, np.concatenate([ubar, ut]), tau=tau)
    c_pol = O.velocity_divergence(cfg, np.concatenate([up.ravel(), np.zeros(3 * len(cells))]), tau=tau)
    assert np.abs(c_enr - c_pol).max() <= 1e-12 * np.abs(c_pol).max()
