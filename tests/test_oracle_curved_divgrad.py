"""Pins of the oracle's pressure gradient term P, velocity divergence term C
and div-div penalty D (Sec. 4.2) on the curved-wall mesh (lower wall y_w = -1 + a cos(2 pi x /
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


def _mapped_y(cfg):
    """The velocity (0, y, 0), y the mapped coordinate at the nodes of every
    cell (no enrichment part), and y per cell as [i][j] node values."""
    n = cfg.k_u + 1
    n3 = n ** 3
    gl = _gl_nodes(n)
    assert np.abs(gl - O.gauss_lobatto(n)).max() < 1e-14
    eta = O.vertex_eta(cfg)
    hx = cfg.Lx / cfg.nx
    u = np.zeros(cfg.n_vel)
    blk = u[:cfg.ncell * 3 * n3].reshape(cfg.ncell, 3, n3)
    Y = {}
    for e in range(cfg.ncell):
        ex, ey = e % cfg.nx, (e // cfg.nx) % cfg.ny
        X, E = np.meshgrid(ex * hx + hx * gl, eta[ey] + (eta[ey + 1] - eta[ey]) * gl, indexing="ij")  # [i][j]
        Y[e] = _curved_y(cfg, X, E)
        blk[e, 1] = np.broadcast_to(Y[e].T[None], (n, n, n)).ravel()   # [m][j][i]
    return u, Y


def _cell_volumes(cfg, Y):
    """|e| = hx hz int_0^1 int_0^1 dy/dxi_y dxi_x dxi_y, y the degree-k_u interpolant of the map."""
    n = cfg.k_u + 1
    gq, wq = np.polynomial.legendre.leggauss(2 * n)
    gq, wq = 0.5 * (gq + 1.0), 0.5 * wq
    vx, dx = _lagrange(_gl_nodes(n), gq)
    return np.array([cfg.Lx / cfg.nx * cfg.Lz / cfg.nz * wq @ np.einsum("ai,bj,ij->ab", vx, dx, Y[e]) @ wq
                     for e in range(cfg.ncell)])


@pytest.mark.parametrize("name", list(CURVED))
def test_divergence_of_the_mapped_coordinate(name):
    cfg = CURVED[name]
    n, npp = cfg.k_u + 1, cfg.k_p + 1
    gl, glp = _gl_nodes(n), _gl_nodes(npp)
    hx, hz = cfg.Lx / cfg.nx, cfg.Lz / cfg.nz
    u, Y = _mapped_y(cfg)
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


@pytest.mark.parametrize("name", list(CURVED))
def test_divdiv_penalty_on_curved_cells(name):
    """tau_D (eq. tauD) of a constant field is |U| |e|^(1/3) dt/Cr; the penalty
    (eq. div-div) vanishes on it, is symmetric, and on the mapped-coordinate
    field (div = 1) its cell-wise energy u^T D_e u is tau_e |e|."""
    cfg = CURVED[name]
    n3 = (cfg.k_u + 1) ** 3
    uY, Y = _mapped_y(cfg)
    vol = _cell_volumes(cfg, Y)
    U = np.array([0.3, -0.7, 1.1])
    uU = _const_velocity(cfg, U)
    td = O.divdiv_tau(cfg, uU, 0.05)
    ref = np.linalg.norm(U) * np.cbrt(vol) * 0.05
    assert np.abs(td - ref).max() <= 1e-13 * ref.max()
    rng = np.random.default_rng(6)
    tau_d = rng.uniform(0.5, 2.0, cfg.ncell)
    u, v = rng.uniform(-1, 1, cfg.n_vel), rng.uniform(-1, 1, cfg.n_vel)
    du, dv = O.divdiv_apply(cfg, u, tau_d), O.divdiv_apply(cfg, v, tau_d)
    assert abs(v @ du - u @ dv) <= 1e-12 * (np.abs(v) @ np.abs(du))
    assert np.abs(O.divdiv_apply(cfg, uU, tau_d)).max() <= 1e-13 * np.abs(du).max()
    dY = O.divdiv_apply(cfg, uY, tau_d)
    en = (uY[:cfg.ncell * 3 * n3] * dY[:cfg.ncell * 3 * n3]).reshape(cfg.ncell, -1).sum(1)
    assert np.abs(en - tau_d * vol).max() <= 1e-12 * (tau_d * vol).max()


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
    u_enr, u_pol = np.concatenate([ubar, ut]), np.concatenate([up.ravel(), np.zeros(3 * len(cells))])
    c_enr = O.velocity_divergence(cfg, u_enr, tau=tau)
    c_pol = O.velocity_divergence(cfg, u_pol, tau=tau)
    assert np.abs(c_enr - c_pol).max() <= 1e-12 * np.abs(c_pol).max()
    # the div-div penalty and tau_D: the same field gives the same values, the
    # enrichment rows are the polynomial rows weighted by psi at the nodes
    t_enr, t_pol = O.divdiv_tau(cfg, u_enr, 0.05, tau=tau), O.divdiv_tau(cfg, u_pol, 0.05, tau=tau)
    assert np.abs(t_enr - t_pol).max() <= 1e-12 * np.abs(t_pol).max()
    tau_d = rng.uniform(0.5, 2.0, cfg.ncell)
    d_enr, d_pol = O.divdiv_apply(cfg, u_enr, tau_d, tau=tau), O.divdiv_apply(cfg, u_pol, tau_d, tau=tau)
    assert np.abs(d_enr[:off] - d_pol[:off]).max() <= 1e-12 * np.abs(d_pol[:off]).max()
    for k, e in enumerate(cells):
        ps = np.array([O.psi_point(cfg, tau, int(e), (gl[B % n], gl[(B // n) % n], gl[B // (n * n)]))[0]
                       for B in range(n3)])
        for c in range(3):
            rows = d_pol[(e * 3 + c) * n3:(e * 3 + c + 1) * n3]
            assert abs(d_enr[off + 3 * k + c] - ps @ rows) <= 1e-12 * (np.abs(ps) @ np.abs(rows))
    # the vorticity right-hand side (v, curl u)_e likewise
    from oracle import step as OS
    b_enr, b_pol = OS.vorticity_rhs(cfg, u_enr, tau), OS.vorticity_rhs(cfg, u_pol, tau)
    assert np.abs(b_enr[:off] - b_pol[:off]).max() <= 1e-12 * np.abs(b_pol[:off]).max()
    for k, e in enumerate(cells):
        ps = np.array([O.psi_point(cfg, tau, int(e), (gl[B % n], gl[(B // n) % n], gl[B // (n * n)]))[0]
                       for B in range(n3)])
        for c in range(3):
            rows = b_pol[(e * 3 + c) * n3:(e * 3 + c + 1) * n3]
            assert abs(b_enr[off + 3 * k + c] - ps @ rows) <= 1e-12 * (np.abs(ps) @ np.abs(rows))


def _numpy_mass(cfg, e, Y, nqx, nqy, psi_k=None):
    """Mass matrix of curved cell e from the map's definition in numpy:
    hx hz sum_q w_q dy/dxi_y(q) phi_i(q) phi_j(q) over an nqx x nqy x nqx Gauss
    rule (phi: the nodal basis, plus psi_k given at that rule's points)."""
    n = cfg.k_u + 1
    gl = _gl_nodes(n)
    gx, wx = np.polynomial.legendre.leggauss(nqx)
    gy, wy = np.polynomial.legendre.leggauss(nqy)
    gx, wx, gy, wy = 0.5 * (gx + 1), 0.5 * wx, 0.5 * (gy + 1), 0.5 * wy
    vx, dx = _lagrange(gl, gx)
    vy, dy = _lagrange(gl, gy)
    dydy = np.einsum("ai,bj,ij->ab", vx, dy, Y[e])                       # [qx][qy]
    w = cfg.Lx / cfg.nx * cfg.Lz / cfg.nz * np.einsum("a,b,c,ab->cba", wx, wy, wx, dydy).ravel()
    V = np.einsum("ai,bj,ck->cbakji", vx, vy, vx).reshape(nqx * nqy * nqx, n ** 3)   # q = qx + nqx (qy + nqy qz)
    Phi = V if psi_k is None else np.hstack([V, np.asarray(psi_k)[:, None]])
    return Phi.T @ (w[:, None] * Phi)


@pytest.mark.parametrize("name", list(CURVED))
def test_mass_matrix_on_curved_cells(name):
    """The velocity mass matrix (M du/dt = -R(u), Sec. 4.1) of a curved cell
    against the numpy matrix with |det J| from the map's definition (the
    cell's rule integrates its polynomial integrand exactly), and M^{-1}."""
    from oracle import project as OP
    cfg = CURVED[name]
    n3 = (cfg.k_u + 1) ** 3
    _, Y = _mapped_y(cfg)
    rng = np.random.default_rng(7)
    x = rng.uniform(-1, 1, cfg.n_vel)
    y = OP.mass_apply(cfg, x, [])
    for e in range(cfg.ncell):
        M = _numpy_mass(cfg, e, Y, 2 * cfg.k_u + 2, 2 * cfg.k_u + 2)
        for c in range(3):
            blk = slice((e * 3 + c) * n3, (e * 3 + c + 1) * n3)
            ref = M @ x[blk]
            assert np.abs(y[blk] - ref).max() <= 1e-13 * np.abs(M).sum(1).max() * np.abs(x[blk]).max()
    xi = OP.inverse_mass(cfg, y, [])
    assert np.abs(xi - x).max() <= 1e-10


def test_mass_matrix_on_curved_enriched_cells():
    """Enriched curved cells: the bordered block (psi row and column) against
    numpy with the oracle's psi at the enriched rule, and M^{-1} M = I within
    eps cond(M)."""
    from oracle import project as OP
    cfg = MeshConfig(nx=4, ny=3, nz=2, wall_amp=0.3, k_u=3, nq_u=5, nq_wn=8, k_p=2, nq_p=3)
    n3 = (cfg.k_u + 1) ** 3
    rng = np.random.default_rng(8)
    tau = rng.uniform(0.2, 2.0, cfg.n_tau)
    cells = O.enriched_cells(cfg)
    psi = O.psi_volume(cfg, cells, tau=tau)
    _, Y = _mapped_y(cfg)
    x = rng.uniform(-1, 1, cfg.n_vel)
    y = OP.mass_apply(cfg, x, psi)
    off = cfg.ncell * 3 * n3
    for k, e in enumerate(cells):
        M = _numpy_mass(cfg, int(e), Y, cfg.nq_u, cfg.nq_wn, psi[k])
        for c in range(3):
            blk = slice((int(e) * 3 + c) * n3, (int(e) * 3 + c + 1) * n3)
            xe = np.concatenate([x[blk], [x[off + 3 * k + c]]])
            ref = M @ xe
            scale = np.abs(M).sum(1).max() * np.abs(xe).max()
            assert np.abs(y[blk] - ref[:n3]).max() <= 1e-13 * scale
            assert abs(y[off + 3 * k + c] - ref[n3]) <= 1e-13 * scale
    xi, cond = OP.inverse_mass(cfg, y, psi, return_cond=True)
    assert np.abs(xi - x).max() <= 64 * 2.0 ** -52 * cond.max() * np.abs(x).max()


def _coordinate_fields(cfg):
    """Nodal x and y (the mapped coordinate) of every cell as [cell][m][j][i] arrays."""
    n = cfg.k_u + 1
    gl = _gl_nodes(n)
    _, Y = _mapped_y(cfg)
    hx = cfg.Lx / cfg.nx
    xs = np.zeros((cfg.ncell, n, n, n))
    ys = np.zeros((cfg.ncell, n, n, n))
    for e in range(cfg.ncell):
        xs[e] = (e % cfg.nx) * hx + hx * gl[None, None, :]
        ys[e] = Y[e].T[None]
    return xs, ys


@pytest.mark.parametrize("name", ["k3", "k5", "k3_enriched"])
def test_projected_vorticity_reproduces_constant_curls(name):
    """omega = M^{-1} (v, curl u) (Sec. 4.2) of (0, x, 0), (y, 0, 0) and
    (0, 0, y), y the mapped coordinate (all in the isoparametric velocity
    space), is the constant curl (0, 0, 1), (0, 0, -1) and (1, 0, 0) at every
    node, with vanishing enrichment coefficients where the cells are enriched."""
    from oracle import step as OS
    cfg = CURVED[name] if name in CURVED else MeshConfig(nx=4, ny=3, nz=2, wall_amp=0.3, k_u=3, nq_u=5, nq_wn=8,
                                                          k_p=2, nq_p=3)
    n3 = (cfg.k_u + 1) ** 3
    xs, ys = _coordinate_fields(cfg)
    tau = np.random.default_rng(9).uniform(0.2, 2.0, cfg.n_tau)
    for comp, field, curl in ((1, xs, (0.0, 0.0, 1.0)), (0, ys, (0.0, 0.0, -1.0)), (2, ys, (1.0, 0.0, 0.0))):
        u = np.zeros(cfg.n_vel)
        u[:cfg.ncell * 3 * n3].reshape(cfg.ncell, 3, n3)[:, comp] = field.reshape(cfg.ncell, n3)
        om = OS.vorticity(cfg, u, tau)
        blk = om[:cfg.ncell * 3 * n3].reshape(cfg.ncell, 3, n3)
        for c in range(3):
            assert np.abs(blk[:, c] - curl[c]).max() <= 1e-11, (comp, c)
        assert np.abs(om[cfg.ncell * 3 * n3:]).max() <= 1e-9 if om.size > cfg.ncell * 3 * n3 else True


@pytest.mark.parametrize("name", ["k3_enriched", "k5"])
def test_neumann_wall_term_on_the_curved_wall(name):
    """Wall term of the pressure equation (eq. bc_d_pres) on the curved mesh,
    summed over each wall cell's pressure block (sum_B N^p_B = 1), so that it
    is a face integral computable from the map:
      (a) constant u, omega = 0: f . int n dA = f_x hz dy_w - f_y hx hz (lower
          wall; n dA = (dy_w/dx, -1, 0) dx dz), f_y hx hz on the upper wall;
      (b) omega = (0, 0, y): curl omega = e_x, so -nu hz dy_w (0 above);
      (c) u = (x, 0, 0): div(u (x) u) = 2 x e_x, so -int 2 x (dy_w/dx) dx dz."""
    from oracle import step as OS
    cfg = CURVED[name] if name in CURVED else MeshConfig(nx=4, ny=3, nz=2, wall_amp=0.3, k_u=3, nq_u=5, nq_wn=8,
                                                          k_p=2, nq_p=3)
    n, p3 = cfg.k_u + 1, (cfg.k_p + 1) ** 3
    n3 = n ** 3
    hx, hz = cfg.Lx / cfg.nx, cfg.Lz / cfg.nz
    gl = _gl_nodes(n)
    tau = np.random.default_rng(10).uniform(0.2, 2.0, cfg.n_tau)
    xs, ys = _coordinate_fields(cfg)
    zero = np.zeros(cfg.n_vel)
    yw = lambda x: -1.0 + cfg.wall_amp * np.cos(2.0 * math.pi * x / cfg.Lx)   # noqa: E731
    gq, wq = np.polynomial.legendre.leggauss(2 * n + 2)
    gq, wq = 0.5 * (gq + 1.0), 0.5 * wq

    def cell_sums(rhs, ey):
        return np.array([[rhs[(ex + cfg.nx * (ey + cfg.ny * ez)) * p3:(ex + cfg.nx * (ey + cfg.ny * ez) + 1) * p3].sum()
                          for ex in range(cfg.nx)] for ez in range(cfg.nz)])

    dyw = np.array([yw((ex + 1) * hx) - yw(ex * hx) for ex in range(cfg.nx)])[None, :]
    # (a)
    f = (0.7, -1.3, 0.4)
    u = _const_velocity(cfg, (0.3, -0.7, 1.1))
    r = OS.pressure_neumann(cfg, [u], [zero], (1.0,), f, tau)
    assert np.abs(cell_sums(r, 0) - (f[0] * hz * dyw - f[1] * hx * hz)).max() <= 1e-12
    assert np.abs(cell_sums(r, cfg.ny - 1) - f[1] * hx * hz).max() <= 1e-12
    # (b)
    om = np.zeros(cfg.n_vel)
    om[:cfg.ncell * 3 * n3].reshape(cfg.ncell, 3, n3)[:, 2] = ys.reshape(cfg.ncell, n3)
    r = OS.pressure_neumann(cfg, [zero], [om], (1.0,), (0.0, 0.0, 0.0), tau)
    assert np.abs(cell_sums(r, 0) + cfg.nu * hz * dyw).max() <= 1e-12 * cfg.nu
    assert np.abs(cell_sums(r, cfg.ny - 1)).max() <= 1e-12 * cfg.nu
    # (c): the interpolated wall y_h(x) of each lower cell, its x-derivative at Gauss points
    ux = np.zeros(cfg.n_vel)
    ux[:cfg.ncell * 3 * n3].reshape(cfg.ncell, 3, n3)[:, 0] = xs.reshape(cfg.ncell, n3)
    r = OS.pressure_neumann(cfg, [ux], [zero], (1.0,), (0.0, 0.0, 0.0), tau)
    _, dl = _lagrange(gl, gq)
    ref = np.zeros((1, cfg.nx))
    for ex in range(cfg.nx):
        dydxi = dl @ yw(ex * hx + hx * gl)                           # d y_h / d xi along the wall face
        ref[0, ex] = -hz * np.sum(wq * 2.0 * (ex * hx + hx * gq) * dydxi)
    assert np.abs(cell_sums(r, 0) - ref).max() <= 1e-12 * np.abs(ref).max()
    assert np.abs(cell_sums(r, cfg.ny - 1)).max() <= 1e-12 * np.abs(ref).max()
