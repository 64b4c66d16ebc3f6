"""GPU element-wise projection step (Sec. 4.2, eq. projectionspat) against
the oracle's dense per-cell solve, through the C ABI.

Per cell, ||x_gpu - x_oracle||_inf <= tol ||x_oracle||_inf with tol = 1e-11 in
cells without enrichment (both sides are direct solves; the kernel's passes
through an orthogonal eigenbasis of the whitened block, accurate to about
1e-13) and max(1e-11, 64 eps cond(M_cell)) in enriched cells, whose mass
blocks have condition numbers up to 1e8 (as for the inverse mass).  Every
enriched cell is also held to a backward error that does not grow with the
conditioning: ||(M+D) x_gpu - b|| <= 2 n eps (||M+D|| ||x_gpu|| + ||M|| ||u^|| +
s ||g||) with b = M u^ - s g and M, D the oracle's blocks from basis values.
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
    "k3": MeshConfig(nx=3, ny=3, nz=2, gamma=1.0, k_u=3, k_p=2, nq_u=5, nq_p=3, nq_wn=8, nu=1.0 / 400),
    "k4": MeshConfig(nx=3, ny=4, nz=2, gamma=1.2, k_u=4, k_p=3, nq_u=7, nq_p=4, nq_wn=8, nu=1.0 / 1000),
    "k2": MeshConfig(nx=3, ny=4, nz=2, gamma=1.3, k_u=2, k_p=1, nq_u=4, nq_p=2, nq_wn=8, nu=1.0 / 800),
    "k5": MeshConfig(nx=2, ny=3, nz=2, gamma=0.8, k_u=5, k_p=4, nq_u=8, nq_p=5, nq_wn=8, nu=1.0 / 600),
    # 9 cells per layer: one full and one partial 8-cell tile at k = 5
    "k5_wide": MeshConfig(nx=3, ny=3, nz=3, gamma=0.8, k_u=5, k_p=4, nq_u=8, nq_p=5, nq_wn=8, nu=1.0 / 600),
    # 20 cells per layer: one full and one partial 16-cell matrix-core tile at k = 3
    "k3_wide": MeshConfig(nx=5, ny=3, nz=4, gamma=1.0, k_u=3, k_p=2, nq_u=5, nq_p=3, nq_wn=8, nu=1.0 / 400),
    "k3_one_sided": MeshConfig(nx=3, ny=3, nz=2, gamma=1.0, k_u=3, k_p=2, nq_u=5, nq_p=3, nq_wn=8, nu=1.0 / 400,
                               enrich_upper=0),
    "k3_two_layers": MeshConfig(nx=3, ny=2, nz=2, gamma=1.0, k_u=3, k_p=2, nq_u=5, nq_p=3, nq_wn=8, nu=1.0 / 400),
    "k3_plain": MeshConfig(nx=3, ny=3, nz=2, gamma=1.1, k_u=3, k_p=2, nq_u=5, nq_p=3, enrich_lower=0,
                           enrich_upper=0),
    "k2_periodic": MeshConfig(nx=3, ny=3, nz=2, k_u=2, k_p=1, nq_u=4, nq_p=2, fully_periodic=1),
    "k3_switch_off": MeshConfig(nx=3, ny=3, nz=2, gamma=1.0, k_u=3, k_p=2, nq_u=5, nq_p=3, nq_wn=8, nu=1.0 / 400,
                                yplus_off=275.0),
}


@pytest.mark.parametrize("name", list(CASES))
def test_projection_step_matches_oracle(name):
    cfg = CASES[name]
    print(f"[gpu] projection step case={name}", flush=True)
    inp = draw_inputs(Workload("ps", cfg, 21, 0.5, 1.5))
    g = np.random.default_rng(22).uniform(-1, 1, cfg.n_vel)
    tau_d = O.divdiv_tau(cfg, inp["u"], 0.05, tau=inp["tau"])
    cells = O.enriched_cells(cfg)
    psi4 = O.psi_volume4(cfg, cells, tau=inp["tau"]) if cells.size else np.zeros((0, 1, 4))
    ref = OP.projection_step(cfg, inp["u"], g, 0.7, tau_d, psi4)
    _, conds = OP.inverse_mass(cfg, inp["u"], psi4[..., 0] if cells.size else np.zeros((0, 1)), return_cond=True)
    mesh = Mesh(cfg, inp["tau"])
    x = mesh.projection_step(torch.tensor(tau_d, device="cuda"), torch.tensor(inp["u"], device="cuda"),
                             torch.tensor(g, device="cuda"), 0.7).cpu().numpy()
    _check(cfg, x, ref, conds, range(cfg.ncell), (inp["u"], g, 0.7, tau_d, psi4))


def _check(cfg, x, ref, conds, check_cells, bwd=None):
    """bwd: (u_hat, g, scale, tau_d, psi4) for the backward-error check of the
    enriched cells."""
    n3 = 3 * (cfg.k_u + 1) ** 3
    off = cfg.ncell * n3
    enr = {int(e): k for k, e in enumerate(O.enriched_cells(cfg))}
    worst = worst_bwd = 0.0
    for e in check_cells:
        e = int(e)
        idx = np.arange(e * n3, (e + 1) * n3)
        k = enr.get(e)
        if k is not None:
            idx = np.concatenate([idx, off + 3 * k + np.arange(3)])
        err = np.abs(x[idx] - ref[idx]).max() / max(np.abs(ref[idx]).max(), 1e-300)
        tol = 1e-11 if k is None else max(1e-11, 64 * EPS * conds[e])
        worst = max(worst, err / tol)
        assert err <= tol, (e, err, tol)
        if k is not None and bwd is not None:
            u_hat, g, scale, tau_d, psi4 = bwd
            M, D = OP.projection_block(cfg, e, tau_d[e], psi4[k])
            rows = idx if M.shape[0] == idx.size else idx[:n3]
            b = M @ u_hat[rows] - scale * g[rows]
            babs = np.abs(M) @ np.abs(u_hat[rows]) + abs(scale) * np.abs(g[rows])
            eta = backward_error(M + D, x[rows], b, babs)
            worst_bwd = max(worst_bwd, eta / EPS)
            assert eta <= 2 * M.shape[0] * EPS, (e, eta / EPS)
    print(f"[gpu]   worst err/tol {worst:.3f}" + (f", worst backward error {worst_bwd:.1f} eps" if bwd else ""),
          flush=True)


def test_projection_step_large_mesh_sampled():
    """The bench mesh, wall cells at y+ ~ 70-120, tau_D,e = s_e h_e dt/Cr as in
    eq. tauD with seeded speeds s_e in [0.5, 1.5], h_e the cube root of the
    cell volume and dt/Cr = 0.05; sampled cells (both corners, enriched ones)
    checked."""
    wl = PRESETS["large"]
    cfg = wl.mesh
    print("[gpu] projection step large mesh", flush=True)
    inp = draw_inputs(wl)
    tau = 1600.0 * inp["tau"]
    rng = np.random.default_rng(25)
    g = rng.uniform(-1, 1, cfg.n_vel)
    eta = O.vertex_eta(cfg)
    hy = np.diff(eta)[(np.arange(cfg.ncell) // cfg.nx) % cfg.ny]
    h_e = np.cbrt(cfg.Lx / cfg.nx * hy * cfg.Lz / cfg.nz)
    tau_d = rng.uniform(0.5, 1.5, cfg.ncell) * h_e * 0.05
    mesh = Mesh(cfg, tau)
    x = mesh.projection_step(torch.tensor(tau_d, device="cuda"), torch.tensor(inp["u"], device="cuda"),
                             torch.tensor(g, device="cuda"), 1.3).cpu().numpy()
    ecells = O.enriched_cells(cfg)
    pick_e = ecells[np.unique(rng.integers(0, ecells.size, 10))]
    cells = np.unique(np.concatenate([rng.integers(0, cfg.ncell, 30), pick_e, [0, cfg.ncell - 1]]))
    enr = {int(e): k for k, e in enumerate(ecells)}
    npts = cfg.nq_u * cfg.nq_wn * cfg.nq_u
    psi4 = np.zeros((ecells.size, npts, 4))
    ek = [enr[int(e)] for e in cells if int(e) in enr]
    psi4[ek] = O.psi_volume4(cfg, ecells[ek], tau=tau)
    ref = OP.projection_step(cfg, inp["u"], g, 1.3, tau_d, psi4, cells=cells)
    _, conds = OP.inverse_mass(cfg, inp["u"], psi4[..., 0], cells=cells, return_cond=True)
    _check(cfg, x, ref, conds, cells, (inp["u"], g, 1.3, tau_d, psi4))


def test_projection_step_rejects_bad_arguments():
    mesh = Mesh(CASES["k3"])
    u = torch.zeros(mesh.n_vel, dtype=torch.float64, device="cuda")
    td = torch.ones(mesh.n_cells, dtype=torch.float64, device="cuda")
    with pytest.raises(DgError) as ei:
        mesh.projection_step(td, u, u.clone(), 1.0, u)
    assert ei.value.code == -1
    curved = Mesh(MeshConfig(nx=4, ny=3, nz=2, wall_amp=0.3, k_u=3, nq_u=5, nq_wn=8, k_p=2, nq_p=3))
    uc = torch.zeros(curved.n_vel, dtype=torch.float64, device="cuda")
    with pytest.raises(DgError) as ei:
        curved.projection_step(torch.ones(curved.n_cells, dtype=torch.float64, device="cuda"), uc, uc.clone(), 1.0)
    assert ei.value.code == -6


def test_projection_step_without_penalty_is_inverse_mass():
    """tau_D = 0 on the bench mesh: (M) x = M u_hat - s g, so x = u_hat - s M^{-1} g
    in every cell (direct per-layer solve, bordered in enriched cells)."""
    wl = PRESETS["large"]
    cfg = wl.mesh
    print("[gpu] projection step, zero penalty, large mesh", flush=True)
    inp = draw_inputs(wl, want=("u", "tau"))
    mesh = Mesh(cfg, 1600.0 * inp["tau"])
    u = torch.tensor(inp["u"], device="cuda")
    g = torch.tensor(np.random.default_rng(26).uniform(-1, 1, cfg.n_vel), device="cuda")
    x = mesh.projection_step(torch.zeros(cfg.ncell, dtype=torch.float64, device="cuda"), u, g, 0.9)
    ref = u - 0.9 * mesh.apply_inverse_mass(g)
    n3 = 3 * (cfg.k_u + 1) ** 3
    regular = np.ones(cfg.ncell, dtype=bool)
    regular[O.enriched_cells(cfg)] = False
    reg = torch.tensor(np.repeat(regular, n3), device="cuda")
    err_reg = ((x[:cfg.ncell * n3][reg] - ref[:cfg.ncell * n3][reg]).abs().max() / ref.abs().max()).item()
    err_all = ((x - ref).abs().max() / ref.abs().max()).item()
    print(f"[gpu]   cells without enrichment {err_reg:.2e}, all {err_all:.2e}", flush=True)
    # regular cells: exact solves; enriched cells: both sides carry the
    # mass block's conditioning (up to ~1e7 here), bound 64 eps cond
    assert err_reg <= 1e-12 and err_all <= 64 * EPS * 1e7


def test_projection_step_follows_wall_shear_update():
    """The cached psi-dependent parts are refreshed by a wall-shear update:
    step, update to a new tau_w, step again -> the oracle on the new psi."""
    cfg = CASES["k3"]
    print("[gpu] projection step after a wall-shear update", flush=True)
    inp = draw_inputs(Workload("ps", cfg, 27, 0.5, 1.5))
    tau2 = 3.0 * inp["tau"]
    g = np.random.default_rng(28).uniform(-1, 1, cfg.n_vel)
    tau_d = O.divdiv_tau(cfg, inp["u"], 0.05, tau=tau2)
    mesh = Mesh(cfg, inp["tau"])
    td, u, gd = (torch.tensor(a, device="cuda") for a in (tau_d, inp["u"], g))
    mesh.projection_step(td, u, gd, 0.7)
    mesh.update_wall_shear(torch.tensor(tau2, device="cuda"))
    x = mesh.projection_step(td, u, gd, 0.7).cpu().numpy()
    cells = O.enriched_cells(cfg)
    psi4 = O.psi_volume4(cfg, cells, tau=tau2)
    ref = OP.projection_step(cfg, inp["u"], g, 0.7, tau_d, psi4)
    _, conds = OP.inverse_mass(cfg, inp["u"], psi4[..., 0], return_cond=True)
    _check(cfg, x, ref, conds, range(cfg.ncell), (inp["u"], g, 0.7, tau_d, psi4))


def test_projection_step_is_repeatable():
    """Two calls on the same inputs give the same bits (fixed-order sums, no atomics)."""
    cfg = CASES["k4"]
    inp = draw_inputs(Workload("ps", cfg, 29, 0.5, 1.5))
    mesh = Mesh(cfg, inp["tau"])
    td = torch.tensor(O.divdiv_tau(cfg, inp["u"], 0.05, tau=inp["tau"]), device="cuda")
    u = torch.tensor(inp["u"], device="cuda")
    g = torch.tensor(np.random.default_rng(30).uniform(-1, 1, cfg.n_vel), device="cuda")
    x1 = mesh.projection_step(td, u, g, 0.7)
    x2 = mesh.projection_step(td, u, g, 0.7)
    assert torch.equal(x1, x2)
