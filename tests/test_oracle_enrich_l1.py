"""Pins of the oracle's degree-1 enrichment weights (no GPU).

Sec. 3.1 eq. enrichment writes the enrichment as psi times a tensor-product
expansion of degree l; l = 1 uses the eight trilinear vertex functions of the
cell, so an enriched cell carries 3 x 8 = 24 enrichment unknowns instead of 3
(Sec. 5.1, the l = 0 / l = 1 comparison).  Two reductions tie the l = 1
residual to separately pinned paths:

- partition of unity: the vertex functions sum to one, so eight equal
  coefficients reproduce the l = 0 field, and the eight enrichment rows of a
  component sum to its l = 0 row;
- polynomial psi: with a vanishing wall shear stress Spalding's psi is y+,
  linear in y, so psi N_B is a polynomial of degree 2 in y and 1 in x, z; for
  k >= 2 the enriched residual then equals the polynomial-only residual of the
  interpolated field, and each enrichment row is the polynomial rows weighted
  by psi N_B at the nodes.
"""
import math

import numpy as np
import pytest

import oracle as O
from oracle import project as OP
from oracle import step as OS
from paper_1705_08813_amd.inputs import MeshConfig, PRESETS, Workload, draw_inputs


def _vertex_fn(b, xi):
    """Trilinear vertex function B = bx + 2 (by + 2 bz) at reference point xi."""
    bits = (b & 1, (b >> 1) & 1, (b >> 2) & 1)
    v = 1.0
    for d in range(3):
        v *= xi[d] if bits[d] else 1.0 - xi[d]
    return v


def test_dof_count_24_per_enriched_cell():
    cfg = PRESETS["tiny"].mesh.with_(enrich_degree=1)
    n3 = (cfg.k_u + 1) ** 3
    assert cfg.n_enr_dofs == 24 * cfg.n_enriched
    assert O.num_dofs(cfg, 0) == cfg.ncell * 3 * n3 + 24 * cfg.n_enriched
    assert O.num_dofs(cfg.with_(enrich_degree=0), 0) == cfg.ncell * 3 * n3 + 3 * cfg.n_enriched
    assert O.num_dofs(cfg.with_(enrich_degree=2), 0) == -1          # only l = 0 and l = 1 exist


CASES_POU = {
    "tiny_spalding": PRESETS["tiny"],
    "k2_vandriest_stretched": Workload("l1a", MeshConfig(nx=3, ny=3, nz=2, gamma=1.3, k_u=2, nq_u=4, nq_wn=8,
                                                          psi_kind=1), 71, 0.5, 1.5),
    "k3_lower_only": Workload("l1b", MeshConfig(nx=2, ny=3, nz=3, gamma=0.7, k_u=3, nq_u=5, nq_wn=8,
                                                 enrich_upper=0), 72, 0.3, 2.0),
}


@pytest.mark.parametrize("conv", [False, True])
@pytest.mark.parametrize("name", list(CASES_POU))
def test_partition_of_unity_reduces_to_l0(name, conv):
    wl = CASES_POU[name]
    cfg0 = wl.mesh
    cfg1 = cfg0.with_(enrich_degree=1)
    inp = draw_inputs(wl)
    f = O.convective_residual if conv else O.velocity_residual
    n = cfg0.ncell * 3 * (cfg0.k_u + 1) ** 3
    ut = inp["u"][n:].reshape(-1, 3)
    u1 = np.concatenate([inp["u"][:n], np.repeat(ut[:, :, None], 8, axis=2).ravel()])
    r0 = f(cfg0, inp["u"], inp["tau"])
    r1 = f(cfg1, u1, inp["tau"])
    scale = np.abs(r0).max()
    assert np.abs(r1[:n] - r0[:n]).max() <= 1e-13 * scale
    rows = r1[n:].reshape(-1, 3, 8)
    assert np.abs(rows.sum(axis=2) - r0[n:].reshape(-1, 3)).max() <= 1e-13 * scale
    # the rows of one cell are not all alike (the weights see the field)
    assert np.abs(rows - rows.mean(axis=2, keepdims=True)).max() > 1e-6 * np.abs(rows).max()


@pytest.mark.parametrize("k,gamma", [(2, 0.0), (3, 1.1)])
def test_l1_enrichment_with_linear_psi_reduces_to_polynomial_path(k, gamma):
    nq = (3 * k) // 2 + 1
    base = MeshConfig(nx=2, ny=3, nz=2, gamma=gamma, k_u=k, nq_u=nq, nq_wn=nq, enrich_degree=1)
    tau_val = 1e-14
    cfg_p = base.with_(enrich_lower=0, enrich_upper=0)
    n = k + 1
    n3 = n ** 3
    rng = np.random.default_rng(10 + k)
    ubar = rng.uniform(-1, 1, base.ncell * 3 * n3)
    s = math.sqrt(tau_val) / base.nu
    eta = O.vertex_eta(base)
    ut = rng.uniform(-1, 1, 24 * base.n_enriched) / (2 * s)    # psi ut = O(1)
    r_e = O.velocity_residual(base, np.concatenate([ubar, ut]), np.full(base.n_tau, tau_val))
    nodes = O.gauss_lobatto(n)
    up = ubar.copy().reshape(base.ncell, 3, n3)
    weights = {}
    enr = 0
    for e in range(base.ncell):
        ey = (e // base.nx) % base.ny
        if ey not in (0, base.ny - 1):
            continue
        pn = np.zeros((8, n3))                                   # psi N_B at the nodes
        for m in range(n):
            for j in range(n):
                for i in range(n):
                    y = eta[ey] + (eta[ey + 1] - eta[ey]) * nodes[j]
                    ps = s * ((y + 1) if ey == 0 else (1 - y))
                    for b in range(8):
                        pn[b, i + n * (j + n * m)] = ps * _vertex_fn(b, (nodes[i], nodes[j], nodes[m]))
        for c in range(3):
            up[e, c] += ut[24 * enr + 8 * c: 24 * enr + 8 * c + 8] @ pn
        weights[e] = (enr, pn)
        enr += 1
    r_p = O.velocity_residual(cfg_p, up.ravel(), None)
    scale = np.abs(r_p).max()
    assert np.abs(r_e[: base.ncell * 3 * n3] - r_p).max() < 1e-12 * scale
    rp = r_p.reshape(base.ncell, 3, n3)
    rt = r_e[base.ncell * 3 * n3:].reshape(-1, 3, 8)
    for e, (i, pn) in weights.items():
        exp = rp[e] @ pn.T                                       # [c][B]
        assert np.abs(rt[i] - exp).max() < 1e-11 * np.abs(exp).max() + 1e-12 * scale * pn.max()


def _rep8(cfg0, v):
    n = cfg0.ncell * 3 * (cfg0.k_u + 1) ** 3
    return np.concatenate([v[:n], np.repeat(v[n:].reshape(-1, 3)[:, :, None], 8, axis=2).ravel()])


def test_l1_mass_partition_of_unity_and_inverse():
    """The l = 1 mass matrix: eight equal coefficients give the l = 0 product
    (polynomial rows equal, enrichment rows summing to the l = 0 row), and
    inverse_mass inverts mass_apply."""
    wl = CASES_POU["k3_lower_only"]
    cfg0 = wl.mesh
    cfg1 = cfg0.with_(enrich_degree=1)
    inp = draw_inputs(wl)
    psi = O.psi_volume(cfg0, O.enriched_cells(cfg0), tau=inp["tau"])
    n = cfg0.ncell * 3 * (cfg0.k_u + 1) ** 3
    y0 = OP.mass_apply(cfg0, inp["u"], psi)
    y1 = OP.mass_apply(cfg1, _rep8(cfg0, inp["u"]), psi)
    scale = np.abs(y0).max()
    assert np.abs(y1[:n] - y0[:n]).max() <= 1e-14 * scale
    assert np.abs(y1[n:].reshape(-1, 3, 8).sum(axis=2) - y0[n:].reshape(-1, 3)).max() <= 1e-14 * scale
    x = np.random.default_rng(90).uniform(-1, 1, cfg1.n_vel)
    back = OP.inverse_mass(cfg1, OP.mass_apply(cfg1, x, psi), psi)
    x_, conds = OP.inverse_mass(cfg1, OP.mass_apply(cfg1, x, psi), psi, return_cond=True)
    # forward error within the blocks' conditioning
    err = np.abs(back - x).max()
    assert err <= 1e3 * np.finfo(float).eps * conds.max() * np.abs(x).max()


def test_l1_helmholtz_oracle_solves_its_equation():
    wl = Workload("l1h", MeshConfig(nx=2, ny=3, nz=2, gamma=1.0, k_u=2, nq_u=4, nq_wn=8, k_p=1, nq_p=2,
                                    nu=1.0 / 400, enrich_degree=1), 91, 0.5, 1.5)
    cfg = wl.mesh
    inp = draw_inputs(wl)
    rng = np.random.default_rng(92)
    b = rng.uniform(-1, 1, cfg.n_vel)
    u_nut = rng.uniform(-1, 1, cfg.n_vel)
    x, its = OS.helmholtz_solve(cfg, u_nut, inp["tau"], 30.0, b)
    r = OS.helmholtz_residual(cfg, u_nut, inp["tau"], 30.0, b, x)
    psi = O.psi_volume(cfg, O.enriched_cells(cfg), tau=inp["tau"])
    assert np.abs(r).max() <= 1e-9 * 30.0 * np.abs(OP.mass_apply(cfg, b, psi)).max()
    assert its > 0


@pytest.mark.parametrize("name", list(CASES_POU))
def test_divgrad_divdiv_partition_of_unity(name):
    """P, C, tau_D and D (Sec. 4.2, eqs. div-div, tauD): eight equal vertex
    coefficients give the l = 0 divergence, tau_D and div-div rows, and the
    eight enrichment rows of a component (P, D) sum to its l = 0 row."""
    wl = CASES_POU[name]
    cfg0 = wl.mesh
    cfg1 = cfg0.with_(enrich_degree=1)
    inp = draw_inputs(wl)
    tau = inp["tau"]
    n = cfg0.ncell * 3 * (cfg0.k_u + 1) ** 3
    u0 = inp["u"]
    u1 = _rep8(cfg0, u0)
    p = np.random.default_rng(73).uniform(-1, 1, cfg0.n_p)
    c0, c1 = O.velocity_divergence(cfg0, u0, tau=tau), O.velocity_divergence(cfg1, u1, tau=tau)
    assert np.abs(c1 - c0).max() <= 1e-13 * np.abs(c0).max()
    t0, t1 = O.divdiv_tau(cfg0, u0, 0.1, tau=tau), O.divdiv_tau(cfg1, u1, 0.1, tau=tau)
    assert np.abs(t1 - t0).max() <= 1e-13 * np.abs(t0).max()
    for f0, f1 in ((O.pressure_gradient(cfg0, p, tau=tau), O.pressure_gradient(cfg1, p, tau=tau)),
                   (O.divdiv_apply(cfg0, u0, t0, tau=tau), O.divdiv_apply(cfg1, u1, t0, tau=tau))):
        scale = np.abs(f0).max()
        assert np.abs(f1[:n] - f0[:n]).max() <= 1e-13 * scale
        rows = f1[n:].reshape(-1, 3, 8)
        assert np.abs(rows.sum(axis=2) - f0[n:].reshape(-1, 3)).max() <= 1e-13 * scale
        assert np.abs(rows - rows.mean(axis=2, keepdims=True)).max() > 1e-6 * np.abs(rows).max()


def _linear_psi_setup(k, gamma, seed):
    """Enriched mesh (l = 1, vanishing tau_w: psi = y+ linear in y), the
    mesh without enrichment, a velocity (ubar, ut) of the first and the
    polynomial field it equals on the second, and psi N_B at the nodes of
    every enriched cell."""
    nq = (3 * k) // 2 + 1
    base = MeshConfig(nx=2, ny=3, nz=2, gamma=gamma, k_u=k, k_p=k - 1, nq_u=nq, nq_wn=nq, nq_p=k,
                      enrich_degree=1)
    tau_val = 1e-14
    cfg_p = base.with_(enrich_lower=0, enrich_upper=0)
    n = k + 1
    n3 = n ** 3
    rng = np.random.default_rng(seed)
    ubar = rng.uniform(-1, 1, base.ncell * 3 * n3)
    s = math.sqrt(tau_val) / base.nu
    eta = O.vertex_eta(base)
    ut = rng.uniform(-1, 1, 24 * base.n_enriched) / (2 * s)
    nodes = O.gauss_lobatto(n)
    up = ubar.copy().reshape(base.ncell, 3, n3)
    weights = {}
    enr = 0
    for e in range(base.ncell):
        ey = (e // base.nx) % base.ny
        if ey not in (0, base.ny - 1):
            continue
        pn = np.zeros((8, n3))
        for m in range(n):
            for j in range(n):
                for i in range(n):
                    y = eta[ey] + (eta[ey + 1] - eta[ey]) * nodes[j]
                    ps = s * ((y + 1) if ey == 0 else (1 - y))
                    for b in range(8):
                        pn[b, i + n * (j + n * m)] = ps * _vertex_fn(b, (nodes[i], nodes[j], nodes[m]))
        for c in range(3):
            up[e, c] += ut[24 * enr + 8 * c: 24 * enr + 8 * c + 8] @ pn
        weights[e] = (enr, pn)
        enr += 1
    return base, cfg_p, np.concatenate([ubar, ut]), up.ravel(), weights, np.full(base.n_tau, tau_val)


def _check_rows(base, f_e, f_p, weights):
    """Polynomial rows equal; each enrichment row is the polynomial rows weighted by psi N_B."""
    n3 = (base.k_u + 1) ** 3
    nb = base.ncell * 3 * n3
    scale = np.abs(f_p).max()
    assert np.abs(f_e[:nb] - f_p).max() < 1e-12 * scale
    fp = f_p.reshape(base.ncell, 3, n3)
    ft = f_e[nb:].reshape(-1, 3, 8)
    for e, (i, pn) in weights.items():
        exp = fp[e] @ pn.T
        assert np.abs(ft[i] - exp).max() < 1e-11 * np.abs(exp).max() + 1e-12 * scale * pn.max()


@pytest.mark.parametrize("k,gamma", [(2, 0.0), (3, 1.1)])
def test_divgrad_divdiv_with_linear_psi_reduce_to_polynomial_path(k, gamma):
    """With psi = y+ every psi N_B is a polynomial of the cell: the l = 1
    divergence and tau_D of (ubar, ut) equal those of the interpolated
    polynomial field on the mesh without enrichment, and P and D give the
    same polynomial rows with enrichment rows weighted by psi N_B at the
    nodes (both sides of D)."""
    base, cfg_p, u_e, u_p, weights, tau = _linear_psi_setup(k, gamma, 20 + k)
    c_e, c_p = O.velocity_divergence(base, u_e, tau=tau), O.velocity_divergence(cfg_p, u_p)
    assert np.abs(c_e - c_p).max() < 1e-12 * np.abs(c_p).max()
    t_e, t_p = O.divdiv_tau(base, u_e, 0.2, tau=tau), O.divdiv_tau(cfg_p, u_p, 0.2)
    assert np.abs(t_e - t_p).max() < 1e-12 * np.abs(t_p).max()
    p = np.random.default_rng(30 + k).uniform(-1, 1, base.n_p)
    _check_rows(base, O.pressure_gradient(base, p, tau=tau), O.pressure_gradient(cfg_p, p), weights)
    _check_rows(base, O.divdiv_apply(base, u_e, t_p, tau=tau), O.divdiv_apply(cfg_p, u_p, t_p), weights)


@pytest.mark.parametrize("name", ["tiny_spalding", "k2_vandriest_stretched"])
def test_vorticity_and_neumann_partition_of_unity(name):
    """The vorticity right-hand side (Sec. 4.2, below eq. ipflux) and the
    wall term of the pressure Neumann data (eq. bc_d_pres): eight equal vertex
    coefficients give the l = 0 results, and the eight enrichment rows of a
    component of the vorticity sum to its l = 0 row."""
    wl = CASES_POU[name]
    cfg0 = wl.mesh
    cfg1 = cfg0.with_(enrich_degree=1)
    inp = draw_inputs(wl)
    tau = inp["tau"]
    n = cfg0.ncell * 3 * (cfg0.k_u + 1) ** 3
    u0 = inp["u"]
    u1 = _rep8(cfg0, u0)
    b0, b1 = OS.vorticity_rhs(cfg0, u0, tau), OS.vorticity_rhs(cfg1, u1, tau)
    scale = np.abs(b0).max()
    assert np.abs(b1[:n] - b0[:n]).max() <= 1e-13 * scale
    rows = b1[n:].reshape(-1, 3, 8)
    assert np.abs(rows.sum(axis=2) - b0[n:].reshape(-1, 3)).max() <= 1e-13 * scale
    om0 = np.random.default_rng(74).uniform(-1, 1, cfg0.n_vel)
    h0 = OS.pressure_neumann(cfg0, [u0], [om0], [1.0], (0.0, 0.3, 0.0), tau)
    h1 = OS.pressure_neumann(cfg1, [u1], [_rep8(cfg0, om0)], [1.0], (0.0, 0.3, 0.0), tau)
    assert np.abs(h1 - h0).max() <= 1e-13 * np.abs(h0).max()


@pytest.mark.parametrize("k,gamma", [(2, 0.0), (3, 1.1)])
def test_vorticity_and_neumann_with_linear_psi_reduce_to_polynomial_path(k, gamma):
    """With psi = y+ the l = 1 vorticity right-hand side has the polynomial
    rows of the interpolated field and enrichment rows weighted by psi N_B at
    the nodes, and the Neumann wall term of (u, omega) equals that of their
    polynomial equivalents."""
    base, cfg_p, u_e, u_p, weights, tau = _linear_psi_setup(k, gamma, 40 + k)
    _check_rows(base, OS.vorticity_rhs(base, u_e, tau), OS.vorticity_rhs(cfg_p, u_p, None), weights)
    _, _, om_e, om_p, _, _ = _linear_psi_setup(k, gamma, 50 + k)
    h_e = OS.pressure_neumann(base, [u_e, u_e], [om_e, om_e], [2.0, -1.0], (0.1, 0.4, 0.0), tau)
    h_p = OS.pressure_neumann(cfg_p, [u_p, u_p], [om_p, om_p], [2.0, -1.0], (0.1, 0.4, 0.0), None)
    assert np.abs(h_e - h_p).max() < 1e-12 * np.abs(h_p).max()


@pytest.mark.parametrize("name", ["tiny_spalding", "k3_lower_only"])
def test_projection_step_l1_meets_its_equation(name):
    """The l = 1 projection step (Sec. 4.2, eq. projectionspat) assembled
    densely per cell satisfies M x + D x = M u_hat - s g with the separately
    pinned l = 1 mass matrix (partition of unity, M^{-1} M = I) and div-div
    penalty (linear-psi reduction), to rounding of the cells' blocks."""
    wl = CASES_POU[name]
    cfg = wl.mesh.with_(enrich_degree=1)
    inp = draw_inputs(wl)
    tau = inp["tau"]
    rng = np.random.default_rng(75)
    u = rng.uniform(-1, 1, cfg.n_vel)
    u_hat = rng.uniform(-1, 1, cfg.n_vel)
    g = rng.uniform(-1, 1, cfg.n_vel)
    s = 0.01
    tau_d = O.divdiv_tau(cfg, u, 0.05, tau=tau)
    cells = O.enriched_cells(cfg)
    psi4 = O.psi_volume4(cfg, cells, tau=tau)
    psi = psi4[:, :, 0]
    x = OP.projection_step(cfg, u_hat, g, s, tau_d, psi4)
    lhs = OP.mass_apply(cfg, x, psi) + O.divdiv_apply(cfg, x, tau_d, tau=tau)
    rhs = OP.mass_apply(cfg, u_hat, psi) - s * g
    scale = np.abs(OP.mass_apply(cfg, np.abs(x), np.abs(psi))).max() + np.abs(rhs).max()
    assert np.abs(lhs - rhs).max() <= 1e-12 * scale
    # the enrichment rows are not trivially zero
    n = cfg.ncell * 3 * (cfg.k_u + 1) ** 3
    assert np.abs(x[n:]).max() > 1e-3 * np.abs(x[:n]).max()


@pytest.mark.parametrize("name", ["tiny_spalding", "k3_lower_only"])
def test_wall_shear_nodes_l1(name):
    """The nodal wall shear stress (Sec. 3.2) with l = 1: eight equal vertex
    coefficients give the l = 0 result, and with psi = y+ the enriched field
    gives that of its polynomial equivalent on the mesh without enrichment."""
    wl = CASES_POU[name]
    cfg0 = wl.mesh
    cfg1 = cfg0.with_(enrich_degree=1)
    inp = draw_inputs(wl)
    t0 = O.wall_shear_nodes(cfg0, inp["u"], tau=inp["tau"])
    t1 = O.wall_shear_nodes(cfg1, _rep8(cfg0, inp["u"]), tau=inp["tau"])
    assert np.abs(t1 - t0).max() <= 1e-13 * np.abs(t0).max()
    base, cfg_p, u_e, u_p, _, tau = _linear_psi_setup(3, 1.1, 60)
    te, tp = O.wall_shear_nodes(base, u_e, tau=tau), O.wall_shear_nodes(cfg_p, u_p)
    assert np.abs(te - tp).max() < 1e-12 * np.abs(tp).max()


def test_l2_projection_l1_same_space_and_reproduction():
    """Eq. l2 with l = 1: the same space reproduces u_old, and with psi_new =
    a psi_old + p (p linear in y, so p N_B stays in Q_k) the field u_bar +
    psi_old sum_B N_B u~_B, which is (u_bar - p sum_B N_B u~_B / a) + psi_new
    sum_B N_B u~_B / a, comes back with u~_new = u~_old / a and that
    polynomial part (p N_B u~_B interpolated at the nodes)."""
    wl = CASES_POU["tiny_spalding"]
    cfg = wl.mesh.with_(enrich_degree=1)
    inp = draw_inputs(wl)
    rng = np.random.default_rng(76)
    u = rng.uniform(-1, 1, cfg.n_vel)
    cells = O.enriched_cells(cfg)
    ps0 = O.psi_volume(cfg, cells, tau=inp["tau"])
    un = OP.project(cfg, u, ps0, ps0)
    assert np.abs(un - u).max() <= 1e-10 * np.abs(u).max()
    a = 1.6
    pts, _ = OP.volume_rule(cfg)
    eta = O.vertex_eta(cfg)
    ps1 = np.empty_like(ps0)
    for k, e in enumerate(cells):
        ey = (e // cfg.nx) % cfg.ny
        y = eta[ey] + (eta[ey + 1] - eta[ey]) * pts[:, 1]
        ps1[k] = a * ps0[k] + 0.3 + 0.2 * y
    un = OP.project(cfg, u, ps0, ps1)
    n = cfg.k_u + 1
    n3 = n ** 3
    off = cfg.ncell * 3 * n3
    nodes = O.gauss_lobatto(n)
    for k, e in enumerate(cells):
        ey = (e // cfg.nx) % cfg.ny
        ut0 = u[off + 24 * k:off + 24 * (k + 1)].reshape(3, 8)
        np.testing.assert_allclose(un[off + 24 * k:off + 24 * (k + 1)], (ut0 / a).ravel(), rtol=1e-9, atol=1e-11)
        pn = np.zeros((8, n3))
        for m in range(n):
            for j in range(n):
                for i in range(n):
                    y = eta[ey] + (eta[ey + 1] - eta[ey]) * nodes[j]
                    for b in range(8):
                        pn[b, i + n * (j + n * m)] = (0.3 + 0.2 * y) * _vertex_fn(b, (nodes[i], nodes[j], nodes[m]))
        for c in range(3):
            exp = u[(e * 3 + c) * n3:(e * 3 + c + 1) * n3] - ut0[c] @ pn / a
            np.testing.assert_allclose(un[(e * 3 + c) * n3:(e * 3 + c + 1) * n3], exp, rtol=0, atol=1e-9)
