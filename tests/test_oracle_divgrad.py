"""Pins of the oracle's pressure gradient term P (velocity test functions) and
velocity divergence term C (pressure test functions) of Sec. 4.2.

- Discrete adjoint: q^T C u = -u^T P q.  Integrating the volume terms by parts
  leaves face terms that cancel between neighbours; with the interior wall
  values of both terms (u+ = u-, p+ = p-) the walls leave the flux of q u . n,
  which vanishes for a q that is zero on the walls (a fully periodic mesh has
  none).  Exact to rounding where the rules integrate div(q u) exactly (cells
  without enrichment).
- A constant velocity has C u = 0: with the interior wall value the wall faces
  close the integration by parts (the mirror value would leave -q u . n).
- Divergence-free fields tangential to the walls have C u = 0: a channel
  profile in the polynomial space, and psi(y) e_x in the enriched layer (psi
  depends on y only for a constant tau_w; integration by parts along x is
  exact for the polynomial q).
- A linear pressure p = y has M^{-1} P p = e_y (no enrichment; M^{-1} is the
  separately pinned inverse mass), and a constant pressure has P p = 0 on the
  x and z components of every row, enrichment rows included.
"""
import numpy as np
import pytest

import oracle as O
from oracle import dense
from oracle import project as OP
from paper_1705_08813_amd.inputs import MeshConfig

PLAIN = [MeshConfig(nx=3, ny=4, nz=2, gamma=1.2, k_u=3, k_p=2, nq_u=5, nq_p=3, enrich_lower=0, enrich_upper=0),
         MeshConfig(nx=2, ny=3, nz=3, gamma=0.0, k_u=4, k_p=3, nq_u=7, nq_p=4, enrich_lower=0, enrich_upper=0),
         MeshConfig(nx=3, ny=3, nz=2, k_u=2, k_p=1, nq_u=4, nq_p=2, fully_periodic=1)]


def _zero_on_walls(cfg, q):
    """q with the node layers on the wall faces (y = -1, y = +1) set to zero."""
    if cfg.fully_periodic:
        return q
    n = cfg.k_p + 1
    qr = q.reshape(cfg.nz, cfg.ny, cfg.nx, n, n, n).copy()   # [ez][ey][ex][k][j][i]
    qr[:, 0, :, :, 0, :] = 0.0
    qr[:, cfg.ny - 1, :, :, n - 1, :] = 0.0
    return qr.reshape(-1)


@pytest.mark.parametrize("cfg", PLAIN)
def test_divergence_is_minus_gradient_transpose(cfg):
    rng = np.random.default_rng(5)
    u = rng.uniform(-1, 1, cfg.n_vel)
    q = _zero_on_walls(cfg, rng.uniform(-1, 1, cfg.n_p))
    tau = np.ones(cfg.n_tau)
    a = q @ O.velocity_divergence(cfg, u, tau=tau)
    b = u @ O.pressure_gradient(cfg, q, tau=tau)
    scale = np.abs(q) @ np.abs(O.velocity_divergence(cfg, np.abs(u), tau=tau))
    assert abs(a + b) <= 1e-13 * max(scale, 1.0), (a, b)
    # and column by column on a few unit vectors (off the walls)
    cand = np.nonzero(_zero_on_walls(cfg, np.ones(cfg.n_p)))[0]
    for i in rng.choice(cand, 4, replace=False):
        ei = np.zeros(cfg.n_p)
        ei[i] = 1.0
        gi = O.pressure_gradient(cfg, ei, tau=tau)
        cu = O.velocity_divergence(cfg, u, tau=tau)
        assert abs(cu[i] + u @ gi) <= 1e-13 * max(np.abs(u) @ np.abs(gi), 1.0)


def _nodal(cfg, f):
    g = dense.lobatto01(cfg.k_u + 1)
    eta = O.vertex_eta(cfg)
    hx, hz = cfg.Lx / cfg.nx, cfg.Lz / cfg.nz
    n3 = (cfg.k_u + 1) ** 3
    u = np.zeros(cfg.n_vel)
    Z, Y, X = np.meshgrid(g, g, g, indexing="ij")
    for e in range(cfg.ncell):
        ex, ey, ez = e % cfg.nx, (e // cfg.nx) % cfg.ny, e // (cfg.nx * cfg.ny)
        x = (ex + X) * hx
        y = eta[ey] + (eta[ey + 1] - eta[ey]) * Y
        z = (ez + Z) * hz
        vals = f(x, y, z)
        for c in range(3):
            u[(e * 3 + c) * n3:(e * 3 + c + 1) * n3] = vals[c].reshape(-1)
    return u


@pytest.mark.parametrize("k", [4, 5])
def test_channel_profile_is_divergence_free(k):
    cfg = MeshConfig(nx=3, ny=4, nz=2, gamma=1.5, k_u=k, k_p=k - 1, nq_u=3 * k // 2 + 1, nq_p=k)
    u = _nodal(cfg, lambda x, y, z: (1 - y ** 2, 0 * y, 0.5 * (1 - y ** 4)))
    c = O.velocity_divergence(cfg, u, tau=np.ones(cfg.n_tau))
    ref = O.velocity_divergence(cfg, np.abs(u), tau=np.ones(cfg.n_tau))
    assert np.abs(c).max() <= 1e-13 * max(np.abs(ref).max(), 1.0)


@pytest.mark.parametrize("cfg", [PLAIN[0], MeshConfig(nx=3, ny=3, nz=2, gamma=1.0, k_u=3, k_p=2, nq_u=5, nq_p=3)])
def test_constant_velocity_has_zero_divergence(cfg):
    u = _nodal(cfg, lambda x, y, z: (0.3 + 0 * y, 1.0 + 0 * y, -0.5 + 0 * y))
    c = O.velocity_divergence(cfg, u, tau=np.ones(cfg.n_tau))
    scale = O.velocity_divergence(cfg, np.abs(u), tau=np.ones(cfg.n_tau))
    # the wall-normal component alone has a nonzero divergence term per cell (sanity of the scale)
    c_y = O.velocity_divergence(cfg, _nodal(cfg, lambda x, y, z: (0 * y, y, 0 * y)), tau=np.ones(cfg.n_tau))
    assert np.abs(c).max() <= 1e-13 * max(np.abs(scale).max(), np.abs(c_y).max())


def test_enrichment_along_x_is_divergence_free():
    # u = psi(y) e_x in both enriched layers (constant tau_w: psi varies with y only)
    cfg = MeshConfig(nx=3, ny=3, nz=2, gamma=1.0, k_u=3, k_p=2, nq_u=5, nq_p=3, nq_wn=8, nu=1.0 / 400)
    u = np.zeros(cfg.n_vel)
    off = cfg.ncell * 3 * (cfg.k_u + 1) ** 3
    u[off::3] = 1.0
    c = O.velocity_divergence(cfg, u, tau=np.full(cfg.n_tau, 0.9))
    # the same field with u~ along y is not divergence free (a check that the test can fail)
    u2 = np.zeros(cfg.n_vel)
    u2[off + 1::3] = 1.0
    c2 = O.velocity_divergence(cfg, u2, tau=np.full(cfg.n_tau, 0.9))
    assert np.abs(c).max() <= 1e-12 * np.abs(c2).max()


def test_linear_pressure_has_unit_gradient():
    cfg = MeshConfig(nx=3, ny=4, nz=2, gamma=1.2, k_u=3, k_p=2, nq_u=5, nq_p=3, enrich_lower=0, enrich_upper=0)
    g = dense.lobatto01(cfg.k_p + 1)
    eta = O.vertex_eta(cfg)
    n3p = (cfg.k_p + 1) ** 3
    p = np.zeros(cfg.n_p)
    Z, Y, X = np.meshgrid(g, g, g, indexing="ij")
    for e in range(cfg.ncell):
        ey = (e // cfg.nx) % cfg.ny
        p[e * n3p:(e + 1) * n3p] = (eta[ey] + (eta[ey + 1] - eta[ey]) * Y).reshape(-1)
    gp = O.pressure_gradient(cfg, p, tau=np.ones(cfg.n_tau))
    x = OP.inverse_mass(cfg, gp, np.zeros((0, 1)))
    n3 = (cfg.k_u + 1) ** 3
    xr = x.reshape(cfg.ncell, 3, n3)
    assert np.abs(xr[:, 0]).max() <= 1e-12 and np.abs(xr[:, 2]).max() <= 1e-12
    assert np.abs(xr[:, 1] - 1.0).max() <= 1e-12


def test_constant_pressure_has_no_tangential_gradient():
    cfg = MeshConfig(nx=3, ny=3, nz=2, gamma=1.0, k_u=3, k_p=2, nq_u=5, nq_p=3, nq_wn=8, nu=1.0 / 400)
    g = O.pressure_gradient(cfg, np.ones(cfg.n_p), tau=np.full(cfg.n_tau, 0.9))
    n3 = (cfg.k_u + 1) ** 3
    off = cfg.ncell * 3 * n3
    gr = g[:off].reshape(cfg.ncell, 3, n3)
    ge = g[off:].reshape(-1, 3)
    scale = np.abs(O.pressure_gradient(cfg, np.ones(cfg.n_p) * 1.0, tau=np.full(cfg.n_tau, 0.9))).max()
    assert np.abs(gr).max() <= 1e-13 * scale          # polynomial rows: all components
    assert np.abs(ge[:, [0, 2]]).max() <= 1e-12 * scale  # enrichment rows: x and z
    assert np.abs(ge[:, 1]).max() > 1e-9 * scale       # y: the rule does not integrate d psi/dy exactly
