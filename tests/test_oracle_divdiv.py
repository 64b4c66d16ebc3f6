"""Pins of the oracle's div-div penalty D(v, u) = (div v, tau_D div u)_e and of
tau_D = ||u||_e h_e dt/Cr (Sec. 4.2, eqs. div-div and tauD).

- tau_D of a constant field is |u| (volume h_e)^(1/3) dt/Cr.
- D u = 0 for divergence-free fields (a channel profile; psi(y) e_x in the
  enriched layers).
- D is symmetric positive semidefinite.
- For u = (0, y, 0) (div u = 1) the polynomial rows are tau_D times the exact
  integrals of d_c N_B, which factor into Gauss-Lobatto weights (the integrals
  of the 1-D nodal basis, here from a 12-point numpy rule) and the jump of N_i
  across the cell: int d_x N_B dV = h_y h_z (N_i(1) - N_i(0)) W_j W_k.
"""
import numpy as np
import pytest

import oracle as O
from oracle import dense
from paper_1705_08813_amd.inputs import MeshConfig, Workload, draw_inputs

CFG = MeshConfig(nx=3, ny=4, nz=2, gamma=1.2, k_u=3, k_p=2, nq_u=5, nq_p=3, nq_wn=8, nu=1.0 / 400)
PLAIN = CFG.with_(enrich_lower=0, enrich_upper=0)


def _nodal(cfg, f):
    g = dense.lobatto01(cfg.k_u + 1)
    eta = O.vertex_eta(cfg)
    hx, hz = cfg.Lx / cfg.nx, cfg.Lz / cfg.nz
    n3 = (cfg.k_u + 1) ** 3
    u = np.zeros(cfg.n_vel)
    Z, Y, X = np.meshgrid(g, g, g, indexing="ij")
    for e in range(cfg.ncell):
        ex, ey, ez = e % cfg.nx, (e // cfg.nx) % cfg.ny, e // (cfg.nx * cfg.ny)
        vals = f((ex + X) * hx, eta[ey] + (eta[ey + 1] - eta[ey]) * Y, (ez + Z) * hz)
        for c in range(3):
            u[(e * 3 + c) * n3:(e * 3 + c + 1) * n3] = np.broadcast_to(vals[c], X.shape).reshape(-1)
    return u


def test_tau_of_constant_field():
    u = _nodal(CFG, lambda x, y, z: (0.6 + 0 * x, -0.8 + 0 * x, 0 * x))
    td = O.divdiv_tau(CFG, u, 0.25, tau=np.ones(CFG.n_tau))
    eta = O.vertex_eta(CFG)
    hy = np.diff(eta)
    h = np.array([(CFG.Lx / CFG.nx * hy[(e // CFG.nx) % CFG.ny] * CFG.Lz / CFG.nz) ** (1 / 3)
                  for e in range(CFG.ncell)])
    np.testing.assert_allclose(td, 1.0 * h * 0.25, rtol=1e-13)


def test_divergence_free_fields_are_not_penalised():
    tau_d = np.random.default_rng(2).uniform(0.5, 2.0, CFG.ncell)
    u = _nodal(CFG, lambda x, y, z: (1 - y ** 2, 0 * y, 0.3 * (1 - y ** 2)))
    d = O.divdiv_apply(CFG, u, tau_d, tau=np.full(CFG.n_tau, 0.9))
    ref = O.divdiv_apply(CFG, _nodal(CFG, lambda x, y, z: (0 * y, y, 0 * y)), tau_d, tau=np.full(CFG.n_tau, 0.9))
    assert np.abs(d).max() <= 1e-13 * np.abs(ref).max()
    ue = np.zeros(CFG.n_vel)
    off = CFG.ncell * 3 * (CFG.k_u + 1) ** 3
    ue[off::3] = 1.0                                        # psi(y) e_x
    assert np.abs(O.divdiv_apply(CFG, ue, tau_d, tau=np.full(CFG.n_tau, 0.9))).max() <= 1e-12 * np.abs(ref).max()


def test_symmetric_positive_semidefinite():
    rng = np.random.default_rng(3)
    tau_d = rng.uniform(0.5, 2.0, CFG.ncell)
    inp = draw_inputs(Workload("dd", CFG, 4, 0.5, 1.5))
    u, v = inp["u"], rng.uniform(-1, 1, CFG.n_vel)
    Du = O.divdiv_apply(CFG, u, tau_d, tau=inp["tau"])
    Dv = O.divdiv_apply(CFG, v, tau_d, tau=inp["tau"])
    assert abs(v @ Du - u @ Dv) <= 1e-12 * abs(v @ Du)
    assert u @ Du > 0 and v @ Dv > 0


@pytest.mark.parametrize("cfg", [PLAIN, CFG])
def test_unit_divergence_closed_form(cfg):
    n = cfg.k_u + 1
    n3 = n ** 3
    tau_d = np.random.default_rng(5).uniform(0.5, 2.0, cfg.ncell)
    d = O.divdiv_apply(cfg, _nodal(cfg, lambda x, y, z: (0 * y, y, 0 * y)), tau_d, tau=np.ones(cfg.n_tau))
    g12, w12 = dense.gauss01(12)
    Nb, _ = dense.basis1d(dense.lobatto01(n), g12)
    W = w12 @ Nb                                            # integrals of the 1-D nodal basis
    jump = np.zeros(n)
    jump[-1], jump[0] = 1.0, -1.0
    eta = O.vertex_eta(cfg)
    hx, hz = cfg.Lx / cfg.nx, cfg.Lz / cfg.nz
    for e in range(cfg.ncell):
        hy = eta[(e // cfg.nx) % cfg.ny + 1] - eta[(e // cfg.nx) % cfg.ny]
        ex_ = tau_d[e] * np.stack([hy * hz * np.einsum("k,j,i->kji", W, W, jump).reshape(-1),
                                   hx * hz * np.einsum("k,j,i->kji", W, jump, W).reshape(-1),
                                   hx * hy * np.einsum("k,j,i->kji", jump, W, W).reshape(-1)])
        np.testing.assert_allclose(d[e * 3 * n3:(e + 1) * 3 * n3], ex_.reshape(-1), rtol=0, atol=1e-12)
