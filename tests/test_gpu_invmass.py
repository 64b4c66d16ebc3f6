"""GPU inverse velocity mass matrix against the oracle's dense per-cell
solve, through the C ABI.

Regular cells (tensor-product blocks, condition numbers below 1e4): 1e-12 of
the largest entry.  Enriched cells: the block of the local basis (N_B, psi)
has condition numbers of 1e6-1e8 where psi is close to a polynomial on the
cell, so any two correct solvers may differ by about eps cond(M) relative to
the cell's solution; each enriched cell is held to 64 eps cond(M_cell) of its
largest entry.  Beside that forward bound every enriched cell is held to a
backward error ||M x_gpu - r|| <= 2 n eps (||M|| ||x_gpu|| + ||r||) per
component (n the block size), M the oracle's block assembled from basis
values: this bound does not grow with cond(M).
"""
import numpy as np
import pytest
import torch

import oracle as O
from oracle import project as OP
from paper_1705_08813_amd import DgError, Mesh
from paper_1705_08813_amd.inputs import PRESETS, MeshConfig, Workload, draw_inputs
from numerics import backward_error

pytestmark = pytest.mark.gpu

EPS = 2.0 ** -52

CASES = {
    "k3": MeshConfig(nx=3, ny=3, nz=2, gamma=1.0, k_u=3, nq_u=5, nq_wn=8, nu=1.0 / 400),
    "k4": MeshConfig(nx=4, ny=4, nz=3, gamma=1.2, k_u=4, nq_u=7, nq_wn=8, nu=1.0 / 1000),
    "k5": MeshConfig(nx=2, ny=3, nz=2, gamma=0.8, k_u=5, nq_u=8, nq_wn=8, k_p=2, nq_p=3, nu=1.0 / 600),
    "k2": MeshConfig(nx=3, ny=4, nz=2, gamma=1.3, k_u=2, nq_u=4, nq_wn=8, k_p=1, nq_p=2, nu=1.0 / 800),
    "k4_lower_only": MeshConfig(nx=3, ny=3, nz=2, gamma=1.0, k_u=4, nq_u=7, nq_wn=8, nu=1.0 / 500, enrich_upper=0),
    "k3_periodic": MeshConfig(nx=3, ny=3, nz=2, k_u=3, nq_u=5, nq_wn=8, fully_periodic=1),
    # a threshold that switches some enriched cells off (their unknowns become 0)
    "k3_switch_off": MeshConfig(nx=3, ny=3, nz=2, gamma=1.0, k_u=3, nq_u=5, nq_wn=8, nu=1.0 / 400, yplus_off=275.0),
}


def _log(msg):
    print(msg, flush=True)


def _check(cfg, x, ref, conds, cells, r=None, psi=None):
    n1 = (cfg.k_u + 1) ** 3
    n3 = 3 * n1
    off = cfg.ncell * n3
    enr = {int(e): k for k, e in enumerate(O.enriched_cells(cfg))}
    worst = worst_bwd = 0.0
    for e in cells:
        idx = np.arange(e * n3, (e + 1) * n3)
        k = enr.get(int(e))
        if k is not None:
            idx = np.concatenate([idx, off + 3 * k + np.arange(3)])
        scale = max(np.abs(ref[idx]).max(), 1e-300)
        err = np.abs(x[idx] - ref[idx]).max() / scale
        tol = 1e-12 if k is None else max(1e-12, 64 * EPS * conds[e])
        worst = max(worst, err / tol)
        assert err <= tol, (int(e), err, tol)
        if k is not None and psi is not None:
            M = OP.mass_block(cfg, e, psi[k])
            for c in range(3):
                rows = np.arange((e * 3 + c) * n1, (e * 3 + c + 1) * n1)
                if M.shape[0] == n1 + 1:
                    rows = np.append(rows, off + 3 * k + c)
                eta = backward_error(M, x[rows], r[rows])
                worst_bwd = max(worst_bwd, eta / EPS)
                assert eta <= 2 * M.shape[0] * EPS, (int(e), c, eta / EPS)
    if psi is not None:
        _log(f"[gpu]   worst backward error {worst_bwd:.1f} eps")
    return worst


@pytest.mark.parametrize("name", list(CASES))
def test_inverse_mass_matches_oracle(name):
    cfg = CASES[name]
    _log(f"[gpu] inverse mass case={name}")
    inp = draw_inputs(Workload("im", cfg, 21, 0.5, 1.5))
    cells = O.enriched_cells(cfg)
    psi = O.psi_volume(cfg, cells, tau=inp["tau"]) if cells.size else np.zeros((0, 1))
    ref, conds = OP.inverse_mass(cfg, inp["u"], psi, return_cond=True)
    mesh = Mesh(cfg, inp["tau"])
    x = mesh.apply_inverse_mass(torch.tensor(inp["u"], device="cuda")).cpu().numpy()
    worst = _check(cfg, x, ref, conds, range(cfg.ncell), inp["u"], psi)
    _log(f"[gpu]   max cond {conds.max():.2e}, worst err/tol {worst:.3f}")
    if name == "k3_switch_off":
        act = O.enrichment_active(cfg, tau=inp["tau"])
        assert 0 < act.sum() < act.size
        n = cfg.ncell * 3 * (cfg.k_u + 1) ** 3
        assert np.all(x[n:][np.repeat(act == 0, 3)] == 0.0)


def test_inverse_mass_in_place_and_after_nodal_update():
    cfg = CASES["k4"]
    inp = draw_inputs(Workload("im", cfg, 22, 0.5, 1.5))
    tn = np.random.default_rng(23).uniform(0.4, 1.6, (2, cfg.nz, cfg.nx))
    mesh = Mesh(cfg, inp["tau"])
    r = torch.tensor(inp["u"], device="cuda")
    x0 = mesh.apply_inverse_mass(r).cpu().numpy()      # fills the cache of the setup psi
    psi0 = O.psi_volume(cfg, O.enriched_cells(cfg), tau=inp["tau"])
    ref0, conds0 = OP.inverse_mass(cfg, inp["u"], psi0, return_cond=True)
    _check(cfg, x0, ref0, conds0, range(cfg.ncell), inp["u"], psi0)
    mesh.update_wall_shear_nodes(torch.tensor(tn, device="cuda"))
    x = mesh.apply_inverse_mass(r)                      # the update invalidates the cache
    y = r.clone()
    mesh.apply_inverse_mass(y, y)
    torch.cuda.synchronize()
    assert torch.equal(x, y)
    psi1 = O.psi_volume(cfg, O.enriched_cells(cfg), tau_nodes=tn)
    ref, conds = OP.inverse_mass(cfg, inp["u"], psi1, return_cond=True)
    _check(cfg, x.cpu().numpy(), ref, conds, range(cfg.ncell), inp["u"], psi1)


def test_inverse_mass_large_mesh_sampled():
    wl = PRESETS["large"]
    cfg = wl.mesh
    _log("[gpu] inverse mass large mesh")
    inp = draw_inputs(wl)
    tau = 1600.0 * inp["tau"]      # wall cells at y+ ~ 70-120
    mesh = Mesh(cfg, tau)
    x = mesh.apply_inverse_mass(torch.tensor(inp["u"], device="cuda")).cpu().numpy()
    rng = np.random.default_rng(24)
    ecells = O.enriched_cells(cfg)
    pick_e = np.unique(rng.integers(0, ecells.size, 12))
    cells = np.unique(np.concatenate([rng.integers(0, cfg.ncell, 40), ecells[pick_e], [0, cfg.ncell - 1]]))
    psi = np.zeros((ecells.size, cfg.nq_u * cfg.nq_wn * cfg.nq_u))
    enr = {int(e): k for k, e in enumerate(ecells)}
    ek = [enr[int(e)] for e in cells if int(e) in enr]
    psi[ek] = O.psi_volume(cfg, ecells[ek], tau=tau)
    ref, conds = OP.inverse_mass(cfg, inp["u"], psi, cells=cells, return_cond=True)
    _check(cfg, x, ref, conds, cells, inp["u"], psi)


# The curved-wall mesh (Sec. 5.2 geometry): non-tensor mass blocks, solved by
# per-cell PCG (and the Schur complement on the psi row in enriched cells).
# Every cell is held to the forward bound (64 eps cond(M) of its largest entry,
# at least 1e-12) and to the backward error 2 n eps of its block.
CURVED = {
    "curved_k3": MeshConfig(nx=4, ny=3, nz=2, wall_amp=0.3, k_u=3, nq_u=5, nq_wn=8, k_p=2, nq_p=3, nu=1.0 / 400),
    "curved_k5": MeshConfig(nx=3, ny=3, nz=2, wall_amp=0.3, gamma=1.2, k_u=5, nq_u=8, nq_wn=8, k_p=4, nq_p=5),
    "curved_k4_two_layers": MeshConfig(nx=3, ny=2, nz=2, wall_amp=0.25, k_u=4, nq_u=7, nq_wn=8, k_p=3, nq_p=4),
    "curved_k2_plain": MeshConfig(nx=4, ny=3, nz=2, wall_amp=0.3, k_u=2, nq_u=4, nq_wn=4, k_p=1, nq_p=2,
                                  enrich_lower=0, enrich_upper=0),
    "curved_k3_lower_only": MeshConfig(nx=3, ny=3, nz=2, wall_amp=0.3, gamma=0.8, k_u=3, nq_u=5, nq_wn=8, k_p=2,
                                       nq_p=3, enrich_upper=0),
}


def _check_curved(cfg, x, r, ref, conds, cells, psi):
    n1 = (cfg.k_u + 1) ** 3
    off = cfg.ncell * 3 * n1
    enr = {int(e): k for k, e in enumerate(O.enriched_cells(cfg))}
    worst = worst_bwd = 0.0
    for e in cells:
        e = int(e)
        k = enr.get(e)
        idx = np.arange(e * 3 * n1, (e + 1) * 3 * n1)
        if k is not None:
            idx = np.concatenate([idx, off + 3 * k + np.arange(3)])
        err = np.abs(x[idx] - ref[idx]).max() / max(np.abs(ref[idx]).max(), 1e-300)
        tol = max(1e-12, 64 * EPS * conds[e])
        worst = max(worst, err / tol)
        assert err <= tol, (e, err, tol)
        M = OP.mass_block(cfg, e, None if k is None else psi[k])
        for c in range(3):
            rows = np.arange((e * 3 + c) * n1, (e * 3 + c + 1) * n1)
            if M.shape[0] == n1 + 1:
                rows = np.append(rows, off + 3 * k + c)
            eta = backward_error(M, x[rows], r[rows])
            worst_bwd = max(worst_bwd, eta / EPS)
            assert eta <= 2 * M.shape[0] * EPS, (e, c, eta / EPS)
    _log(f"[gpu]   max cond {conds.max():.2e}, worst err/tol {worst:.3f}, worst backward error {worst_bwd:.1f} eps")


@pytest.mark.parametrize("name", list(CURVED))
def test_curved_inverse_mass_matches_oracle(name):
    cfg = CURVED[name]
    _log(f"[gpu] curved inverse mass case={name}")
    inp = draw_inputs(Workload("imc", cfg, 25, 0.2, 2.0))
    cells = O.enriched_cells(cfg)
    psi = O.psi_volume(cfg, cells, tau=inp["tau"]) if cells.size else np.zeros((0, 1))
    ref, conds = OP.inverse_mass(cfg, inp["u"], psi, return_cond=True)
    mesh = Mesh(cfg, inp["tau"])
    r = torch.tensor(inp["u"], device="cuda")
    xt = mesh.apply_inverse_mass(r)
    y = r.clone()
    mesh.apply_inverse_mass(y, y)                       # in place
    torch.cuda.synchronize()
    assert torch.equal(xt, y)
    _check_curved(cfg, xt.cpu().numpy(), inp["u"], ref, conds, range(cfg.ncell), psi)


def test_curved_inverse_mass_workload_sampled():
    """The 48 x 24 x 24, k = 5 curved workload on sampled cells (wall rows included)."""
    wl = PRESETS["curved"]
    cfg = wl.mesh
    _log("[gpu] curved inverse mass 48x24x24")
    inp = draw_inputs(wl)
    mesh = Mesh(cfg, inp["tau"])
    x = mesh.apply_inverse_mass(torch.tensor(inp["u"], device="cuda")).cpu().numpy()
    rng = np.random.default_rng(26)
    ecells = O.enriched_cells(cfg)
    pick_e = np.unique(rng.integers(0, ecells.size, 6))
    cells = np.unique(np.concatenate([rng.integers(0, cfg.ncell, 10), ecells[pick_e], [0, cfg.ncell - 1]]))
    psi = np.zeros((ecells.size, cfg.nq_u * cfg.nq_wn * cfg.nq_u))
    enr = {int(e): k for k, e in enumerate(ecells)}
    ek = [enr[int(e)] for e in cells if int(e) in enr]
    psi[ek] = O.psi_volume(cfg, ecells[ek], tau=inp["tau"])
    ref, conds = OP.inverse_mass(cfg, inp["u"], psi, cells=cells, return_cond=True)
    _check_curved(cfg, x, inp["u"], ref, conds, cells, psi)
