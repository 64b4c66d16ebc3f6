"""Pins of the oracle's cell-wise L2 projection (Sec. 3.2, eq. l2) and of the
switch-off rule of the enrichment (Sec. 3.2: off while every quadrature point
of the wall cell has y+ below a threshold).

The projection is checked against closed forms that do not go through the
oracle's nodal basis or dense solve: a field already in the new space is
reproduced; switching the enrichment off leaves the L2 projection of u_old
onto polynomials (computed here by weighted least squares in monomials);
switching it on keeps the polynomial part; and the enrichment coefficient
equals the Schur-complement form u~_new = u~_old <r_new, r_old> / <r_new, r_new>
with r = psi - P psi, P the polynomial L2 projection.
"""
import numpy as np
import pytest

import oracle as O
from oracle import project as OP
from paper_1705_08813_amd.inputs import MeshConfig, Workload, draw_inputs

CFG = MeshConfig(nx=3, ny=3, nz=2, gamma=1.0, k_u=3, nq_u=5, nq_wn=8, nu=1.0 / 400)
WL = Workload("proj", CFG, 31, 0.5, 1.5)


def _inputs(cfg=CFG, seed=31):
    wl = Workload("p", cfg, seed, 0.5, 1.5)
    return draw_inputs(wl)


def _psi(cfg, tau=None, tau_nodes=None):
    return O.psi_volume(cfg, O.enriched_cells(cfg), tau=tau, tau_nodes=tau_nodes)


def _gl_nodes(n):
    # Gauss-Lobatto nodes on [0,1] from numpy's Legendre polynomial (independent of the oracle)
    inner = np.polynomial.legendre.Legendre.basis(n - 1).deriv().roots()
    return 0.5 * (np.concatenate([[-1.0], np.sort(np.real(inner)), [1.0]]) + 1.0)


def _mono(cfg, pts):
    """Monomials x^a y^b z^c, a, b, c <= k, at the points: (npts, (k+1)^3)."""
    n = cfg.k_u + 1
    cols = []
    for c in range(n):
        for b in range(n):
            for a in range(n):
                cols.append(pts[:, 0] ** a * pts[:, 1] ** b * pts[:, 2] ** c)
    return np.stack(cols, axis=1)


def _nodes_xyz(cfg):
    g = _gl_nodes(cfg.k_u + 1)
    Z, Y, X = np.meshgrid(g, g, g, indexing="ij")        # B = i + n (j + n m)
    return np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)


def _poly_fit(cfg, f, pts, w):
    """Weighted least-squares (L2) projection of point values f onto Q_k:
    returns (values at the points, values at the Gauss-Lobatto nodes)."""
    A = _mono(cfg, pts)
    sw = np.sqrt(w)
    coef = np.linalg.lstsq(A * sw[:, None], f * sw, rcond=None)[0]
    return A @ coef, _mono(cfg, _nodes_xyz(cfg)) @ coef


def _blocks(cfg, u):
    n3 = (cfg.k_u + 1) ** 3
    off = cfg.ncell * 3 * n3
    return u[:off].reshape(cfg.ncell, 3, n3), u[off:].reshape(-1, 3)


def test_same_space_is_identity():
    inp = _inputs()
    ps = _psi(CFG, tau=inp["tau"])
    un = OP.project(CFG, inp["u"], ps, ps)
    assert np.abs(un - inp["u"]).max() <= 1e-11 * np.abs(inp["u"]).max()


def test_regular_cells_unchanged():
    inp = _inputs()
    ps0 = _psi(CFG, tau=inp["tau"])
    ps1 = _psi(CFG, tau=inp["tau"] * 1.7)
    un = OP.project(CFG, inp["u"], ps0, ps1)
    ub0, _ = _blocks(CFG, inp["u"])
    ub1, _ = _blocks(CFG, un)
    cells = set(O.enriched_cells(CFG).tolist())
    for e in range(CFG.ncell):
        if e not in cells:
            assert np.array_equal(ub0[e], ub1[e])


def test_field_already_in_new_space_is_reproduced():
    # psi_new = a psi_old + p with p in Q_k: u_old = u_bar + psi_old u~ = (u_bar - p u~/a) + psi_new u~/a
    inp = _inputs()
    pts, _ = OP.volume_rule(CFG)
    ps0 = _psi(CFG, tau=inp["tau"])
    a = 1.6
    p = lambda X: 0.3 + 0.2 * X[:, 1] - 0.15 * X[:, 0] * X[:, 2] + 0.05 * X[:, 0] ** 3 * X[:, 1] ** 2
    ps1 = a * ps0 + p(pts)[None, :]
    un = OP.project(CFG, inp["u"], ps0, ps1)
    ub0, ut0 = _blocks(CFG, inp["u"])
    ub1, ut1 = _blocks(CFG, un)
    pn = p(_nodes_xyz(CFG))
    for k, e in enumerate(O.enriched_cells(CFG)):
        np.testing.assert_allclose(ut1[k], ut0[k] / a, rtol=1e-10, atol=1e-12)
        for c in range(3):
            np.testing.assert_allclose(ub1[e, c], ub0[e, c] - pn * ut0[k, c] / a, rtol=0, atol=1e-10)


def test_switch_off_leaves_polynomial_projection():
    inp = _inputs()
    pts, w = OP.volume_rule(CFG)
    ps0 = _psi(CFG, tau=inp["tau"])
    un = OP.project(CFG, inp["u"], ps0, np.zeros_like(ps0))
    ub0, ut0 = _blocks(CFG, inp["u"])
    ub1, ut1 = _blocks(CFG, un)
    assert np.all(ut1 == 0.0)
    for k, e in enumerate(O.enriched_cells(CFG)):
        _, pnod = _poly_fit(CFG, ps0[k], pts, w)
        for c in range(3):
            np.testing.assert_allclose(ub1[e, c], ub0[e, c] + ut0[k, c] * pnod, rtol=0, atol=1e-9)


def test_switch_on_keeps_polynomial_part():
    inp = _inputs()
    ps1 = _psi(CFG, tau=inp["tau"])
    un = OP.project(CFG, inp["u"], np.zeros_like(ps1), ps1)
    ub0, _ = _blocks(CFG, inp["u"])
    ub1, ut1 = _blocks(CFG, un)
    assert np.abs(ut1).max() <= 1e-12
    cells = O.enriched_cells(CFG)
    assert np.abs(ub1[cells] - ub0[cells]).max() <= 1e-10 * np.abs(ub0).max()


@pytest.mark.parametrize("nodal", [False, True])
def test_enrichment_coefficient_schur_form(nodal):
    inp = _inputs()
    pts, w = OP.volume_rule(CFG)
    if nodal:
        tn0 = np.random.default_rng(1).uniform(0.5, 1.5, (2, CFG.nz, CFG.nx))
        ps0 = _psi(CFG, tau_nodes=tn0)
        ps1 = _psi(CFG, tau_nodes=tn0 * np.random.default_rng(2).uniform(0.6, 1.8, tn0.shape))
    else:
        ps0 = _psi(CFG, tau=inp["tau"])
        ps1 = _psi(CFG, tau=inp["tau"][::-1].copy())
    un = OP.project(CFG, inp["u"], ps0, ps1)
    ub0, ut0 = _blocks(CFG, inp["u"])
    ub1, ut1 = _blocks(CFG, un)
    for k, e in enumerate(O.enriched_cells(CFG)):
        p0q, p0n = _poly_fit(CFG, ps0[k], pts, w)
        p1q, p1n = _poly_fit(CFG, ps1[k], pts, w)
        r0, r1 = ps0[k] - p0q, ps1[k] - p1q
        ratio = np.sum(w * r1 * r0) / np.sum(w * r1 * r1)
        np.testing.assert_allclose(ut1[k], ut0[k] * ratio, rtol=1e-8, atol=1e-12)
        for c in range(3):
            np.testing.assert_allclose(ub1[e, c], ub0[e, c] + ut0[k, c] * p0n - ut1[k, c] * p1n, rtol=0,
                                       atol=1e-8)


def test_projection_does_not_increase_l2_norm():
    inp = _inputs()
    pts, w = OP.volume_rule(CFG)
    V = OP.basis_at(CFG, pts)
    ps0 = _psi(CFG, tau=inp["tau"])
    ps1 = _psi(CFG, tau=inp["tau"] * 3.0)
    un = OP.project(CFG, inp["u"], ps0, ps1)
    ub0, ut0 = _blocks(CFG, inp["u"])
    ub1, ut1 = _blocks(CFG, un)
    for k, e in enumerate(O.enriched_cells(CFG)):
        for c in range(3):
            f0 = V @ ub0[e, c] + ps0[k] * ut0[k, c]
            f1 = V @ ub1[e, c] + ps1[k] * ut1[k, c]
            assert np.sum(w * f1 * f1) <= np.sum(w * f0 * f0) * (1 + 1e-12)
            # and the difference is orthogonal to the new solution (Pythagoras)
            assert abs(np.sum(w * f1 * (f0 - f1))) <= 1e-10 * np.sum(w * f0 * f0)


# ---- switch-off rule ----------------------------------------------------------

def _top_distance(cfg, wall):
    """Largest wall distance among the enriched volume points of a wall cell:
    the wall-normal Gauss point farthest from the wall (numpy's rule)."""
    g = 0.5 * (np.polynomial.legendre.leggauss(cfg.nq_wn)[0] + 1.0)
    if cfg.gamma > 0:
        t = np.array([0, 1, cfg.ny - 1, cfg.ny]) / cfg.ny
        y = np.tanh(cfg.gamma * (2 * t - 1)) / np.tanh(cfg.gamma)
    else:
        y = np.array([0, 1, cfg.ny - 1, cfg.ny]) * 2.0 / cfg.ny - 1.0
    h0, h1 = y[1] - y[0], y[3] - y[2]
    return h0 * g.max() if wall == 0 else h1 * (1.0 - g.min())


@pytest.mark.parametrize("side", [-1, 1])
def test_switch_off_threshold_closed_form(side):
    # constant tau_w: the cell's largest y+ is y_top sqrt(tau)/nu; tau a hair
    # below the threshold switches every cell off, a hair above switches it on
    cfg = CFG.with_(yplus_off=30.0)
    yt = _top_distance(cfg, 0)
    assert abs(yt - _top_distance(cfg, 1)) <= 1e-14   # symmetric grading
    tau_c = (30.0 * cfg.nu / yt) ** 2
    tau = np.full(cfg.n_tau, tau_c * (1 + side * 1e-9))
    act = O.enrichment_active(cfg, tau=tau)
    assert act.size == cfg.n_enriched and np.all(act == (1 if side > 0 else 0))
    # the nodal field of the same constant decides the same way
    tn = np.full((2, cfg.nz, cfg.nx), tau_c * (1 + side * 1e-9))
    assert np.all(O.enrichment_active(cfg, tau_nodes=tn) == act)
    # no threshold: always on
    assert np.all(O.enrichment_active(CFG, tau=tau) == 1)


def test_switch_off_is_per_cell_and_uses_the_largest_point():
    cfg = CFG.with_(yplus_off=30.0)
    yt = _top_distance(cfg, 0)
    tau_c = (30.0 * cfg.nu / yt) ** 2
    nq = cfg.nq_u
    tau = np.full((2, cfg.nz, cfg.nx, nq, nq), 0.5 * tau_c)
    tau[0, 1, 2, 3, 1] = 1.01 * tau_c      # one column of one lower-wall cell above
    act = O.enrichment_active(cfg, tau=tau.ravel())
    cells = O.enriched_cells(cfg)
    on = [k for k in range(cells.size) if act[k]]
    assert len(on) == 1
    e = cells[on[0]]
    assert (e % cfg.nx, (e // cfg.nx) % cfg.ny, e // (cfg.nx * cfg.ny)) == (2, 0, 1)


def test_switched_off_cells_have_zero_psi_and_polynomial_residual():
    cfg = CFG.with_(yplus_off=1e6)           # every cell off
    inp = _inputs()
    ps = _psi(cfg, tau=inp["tau"])
    assert np.all(ps == 0.0)
    r_off = O.velocity_residual(cfg, inp["u"], inp["tau"])
    u0 = inp["u"].copy()
    n3 = (cfg.k_u + 1) ** 3
    u0[cfg.ncell * 3 * n3:] = 0.0
    r_on = O.velocity_residual(CFG, u0, inp["tau"])
    off = cfg.ncell * 3 * n3
    assert np.all(r_off[off:] == 0.0)
    np.testing.assert_allclose(r_off[:off], r_on[:off], rtol=0, atol=1e-13 * np.abs(r_on[:off]).max())
