"""Pins of the oracle's wall-shear pipeline (Sec. 3.2): the nodal wall shear
stress tau_w,B = ||int N_B tau_w dA|| / int N_B dA with tau_w = nu (grad u) n,
and psi with the bilinear nodal tau_w,h and the grad tau_w term of the chain
rule.  Every expected value comes from a closed form or a finite difference,
none from the oracle itself."""
import math

import numpy as np
import pytest

import oracle as O
from paper_1705_08813_amd.inputs import MeshConfig


def _nodes_xyz(cfg):
    """Physical coordinates of every velocity node of a flat mesh, [cell][B][3]."""
    n = cfg.k_u + 1
    gl = O.gauss_lobatto(n)
    eta = O.vertex_eta(cfg)
    hx, hz = cfg.Lx / cfg.nx, cfg.Lz / cfg.nz
    X = np.zeros((cfg.ncell, n ** 3, 3))
    for e in range(cfg.ncell):
        ex, ey, ez = e % cfg.nx, (e // cfg.nx) % cfg.ny, e // (cfg.nx * cfg.ny)
        for m in range(n):
            for j in range(n):
                for i in range(n):
                    B = i + n * (j + n * m)
                    X[e, B] = (ex * hx + gl[i] * hx, eta[ey] + (eta[ey + 1] - eta[ey]) * gl[j], ez * hz + gl[m] * hz)
    return X


def _velocity(cfg, fx, enr=None):
    """Velocity vector with u_x = fx(x, y, z) at the nodes, u_y = u_z = 0, and
    enrichment coefficients enr [enriched cell][3] (zero if None)."""
    n3 = (cfg.k_u + 1) ** 3
    X = _nodes_xyz(cfg)
    u = np.zeros(O.num_dofs(cfg, 0))
    poly = u[: cfg.ncell * 3 * n3].reshape(cfg.ncell, 3, n3)
    poly[:, 0, :] = fx(X[..., 0], X[..., 1], X[..., 2])
    if enr is not None:
        u[cfg.ncell * 3 * n3:] = np.asarray(enr).reshape(-1)
    return u


CFG = MeshConfig(nx=5, ny=4, nz=3, gamma=1.3, k_u=2, nq_u=4, nq_wn=5, k_p=1, nq_p=2, nu=1.0 / 395.0)


def test_linear_profile_gives_nu_times_slope():
    # u_x = a y + b: (grad u) n = -a (lower) / +a (upper) in x; |tau_w| = nu a everywhere
    a, b = 3.7, 0.4
    u = _velocity(CFG, lambda x, y, z: a * y + b)
    tau = np.full(CFG.n_tau, 0.8)
    t = O.wall_shear_nodes(CFG, u, tau=tau)
    assert t.shape == (2, CFG.nz, CFG.nx)
    assert np.abs(t - CFG.nu * a).max() <= 1e-13 * CFG.nu * a


def test_hat_average_of_a_linear_shear_is_the_nodal_value():
    # u_x = (b + c x)(y + 1) - (b + c x) on the upper... use d u_x / d y = b + c x on both walls:
    # the hat-weighted average of a linear function on a uniform grid is its value at the node
    # (interior nodes; the periodic seam mixes x = 0 and x = Lx)
    b, c = 2.0, 0.15
    u = _velocity(CFG, lambda x, y, z: (b + c * x) * y)
    t = O.wall_shear_nodes(CFG, u, tau=np.ones(CFG.n_tau))
    hx = CFG.Lx / CFG.nx
    for w in range(2):
        for iz in range(CFG.nz):
            for ix in range(1, CFG.nx):
                assert abs(t[w, iz, ix] - CFG.nu * (b + c * ix * hx)) <= 1e-13, (w, iz, ix)
        # seam node: the two half-hats see x just below Lx and just above 0
        seam = CFG.nu * (b + c * CFG.Lx / 2)
        assert np.abs(t[w, :, 0] - seam).max() <= 1e-13


def test_enrichment_part_of_the_wall_gradient():
    # u_bar = 0, u~ = (alpha, 0, 0) in the lower enriched layer: d(psi u~)/dy at the wall is
    # alpha U'(0) sqrt(tau_w)/nu with U'(0) = 1 for both laws, so |tau_w| = alpha sqrt(tau_w)
    alpha, tau0 = 0.9, 1.7
    ne = CFG.nx * CFG.nz * 2
    enr = np.zeros((ne, 3))
    lower = [k for k in range(ne) if (k // CFG.nx) % 2 == 0]   # slot 0 = lower wall
    enr[lower, 0] = alpha
    for kind in (0, 1):
        cfg = CFG.with_(psi_kind=kind)
        u = _velocity(cfg, lambda x, y, z: 0 * x, enr)
        t = O.wall_shear_nodes(cfg, u, tau=np.full(cfg.n_tau, tau0))
        assert np.abs(t[0] - alpha * math.sqrt(tau0)).max() <= 1e-13
        assert np.abs(t[1]).max() == 0.0


def _tau_nodes(cfg):
    hx, hz = cfg.Lx / cfg.nx, cfg.Lz / cfg.nz
    xs = np.arange(cfg.nx) * hx
    zs = np.arange(cfg.nz) * hz
    t = np.zeros((2, cfg.nz, cfg.nx))
    for w in range(2):
        t[w] = 1.2 + 0.4 * np.sin(2 * np.pi * xs / cfg.Lx)[None, :] + 0.2 * np.cos(2 * np.pi * zs / cfg.Lz + 0.7)[:, None] \
            + 0.1 * w
    return t


@pytest.mark.parametrize("kind", [0, 1])
def test_nodal_psi_gradient_matches_finite_differences(kind):
    # grad psi = U'(y+) (sqrt(tau)/nu grad y_h + y_h/(2 nu sqrt(tau)) grad tau): central
    # differences of psi in the reference coordinates, mapped by the cell sizes
    cfg = CFG.with_(psi_kind=kind)
    tn = _tau_nodes(cfg)
    eta = O.vertex_eta(cfg)
    hx, hz = cfg.Lx / cfg.nx, cfg.Lz / cfg.nz
    for e in (1, cfg.nx * cfg.ny + 3, cfg.nx * (cfg.ny - 1) + 2):   # lower and upper enriched cells
        ey = (e // cfg.nx) % cfg.ny
        hy = eta[ey + 1] - eta[ey]
        xi = np.array([0.37, 0.61, 0.23])
        g = O.psi_point_nodal(cfg, tn, e, xi)[1:]
        h = 1e-5
        fd = []
        for d, hd in enumerate((hx, hy, hz)):
            xp, xm = xi.copy(), xi.copy()
            xp[d] += h
            xm[d] -= h
            fd.append((O.psi_point_nodal(cfg, tn, e, xp)[0] - O.psi_point_nodal(cfg, tn, e, xm)[0]) / (2 * h * hd))
        fd = np.array(fd)
        assert np.abs(g - fd).max() <= 1e-6 * np.abs(fd).max(), (e, g, fd)
        # on flat walls grad y_h has no x or z part: these components come from the grad tau term alone
        assert abs(g[0]) > 1e-3 and abs(g[2]) > 1e-3


def test_constant_nodal_field_equals_pointwise_field():
    tau0 = 1.3
    tn = np.full((2, CFG.nz, CFG.nx), tau0)
    tp = np.full(CFG.n_tau, tau0)
    rng = np.random.default_rng(4)
    for e in (0, CFG.nx * (CFG.ny - 1)):
        for _ in range(3):
            xi = rng.uniform(0, 1, 3)
            a = O.psi_point(CFG, tp, e, xi)
            b = O.psi_point_nodal(CFG, tn, e, xi)
            assert np.array_equal(a[:2], b[:2]) and abs(a[2] - b[2]) <= 1e-15 * abs(a[2]) and b[1] == 0.0
    u = rng.uniform(-1, 1, O.num_dofs(CFG, 0))
    r1 = O.velocity_residual(CFG, u, tp)
    r2 = O.velocity_residual_nodal(CFG, u, tn)
    assert np.abs(r1 - r2).max() <= 1e-13 * np.abs(r1).max()
