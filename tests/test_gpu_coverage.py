"""Every flat-mesh entry point of the library on every compiled (degree,
rule) combination, with both walls enriched, without enrichment, and fully
periodic: each call must be accepted and give finite output.  (Parity with
the oracle is the business of the other GPU tests; this one guards the
dispatch tables, one of which once refused k = 4 meshes without enrichment
because their unused wall-normal rule differed from the regular one.)
"""
import numpy as np
import pytest
import torch

from paper_1705_08813_amd import Mesh
from paper_1705_08813_amd.inputs import MeshConfig

pytestmark = pytest.mark.gpu

# (k_u + 1, nq_u, nq_wn) as compiled for the velocity operators
COMBOS = [(3, 4, 8), (3, 4, 4), (4, 4, 8), (4, 5, 8), (4, 5, 5), (5, 7, 8), (6, 8, 8)]
KINDS = {
    "enriched": dict(),
    "plain": dict(enrich_lower=0, enrich_upper=0),
    "periodic": dict(fully_periodic=1),
}


def _finite(t):
    return bool(torch.isfinite(t).all())


@pytest.mark.parametrize("kind", list(KINDS))
@pytest.mark.parametrize("combo", COMBOS, ids=[f"np{a}_nq{b}_nw{c}" for a, b, c in COMBOS])
def test_every_entry_point_accepts_the_combination(combo, kind):
    npu, nq, nqw = combo
    cfg = MeshConfig(nx=2, ny=3, nz=2, gamma=0.8, k_u=npu - 1, nq_u=nq, nq_wn=nqw, k_p=npu - 2, nq_p=npu - 1,
                     nu=1.0 / 400, **KINDS[kind])
    print(f"[gpu] coverage k_u={cfg.k_u} nq_u={nq} nq_wn={nqw} {kind}", flush=True)
    rng = np.random.default_rng(npu * 10 + nq)
    tau = rng.uniform(0.5, 1.5, cfg.n_tau)
    mesh = Mesh(cfg, tau)
    u = torch.tensor(0.3 * rng.uniform(-1, 1, cfg.n_vel), device="cuda")
    p = torch.tensor(rng.uniform(-1, 1, cfg.n_p), device="cuda")
    outs = [mesh.apply_velocity_residual(u), mesh.apply_convective(u), mesh.apply_velocity_residual(u.float()),
            mesh.apply_poisson(p), mesh.poisson_diagonal(), mesh.apply_inverse_mass(u),
            mesh.apply_pressure_gradient(p), mesh.apply_velocity_divergence(u), mesh.vorticity(u)]
    td = mesh.divdiv_tau(u, 0.05)
    outs += [td, mesh.apply_divdiv(td, u), mesh.projection_step(td, u, mesh.apply_pressure_gradient(p), 1e-3)]
    nut = mesh.eddy_viscosity(u) if cfg.n_enriched else None
    outs.append(mesh.apply_viscous_multiscale(nut, u))
    x, hst = mesh.solve_helmholtz(nut, 300.0, u, rtol=1e-10)
    outs.append(x)
    if not cfg.fully_periodic:
        outs.append(mesh.wall_shear_nodes(u))
        outs.append(mesh.project_velocity(u))
        outs.append(mesh.pressure_neumann([u], [mesh.vorticity(u)], (1.0,)))
    xs, sst = mesh.solve_poisson(p, sp=mesh.solve_params(rtol=1e-10))
    outs.append(xs)
    sp = mesh.step_params(1e-3, order=1)
    pp = torch.zeros_like(p)
    un, pp, st = mesh.dual_splitting_step(sp, u, None, pp)
    outs += [un, pp]
    assert all(_finite(o) for o in outs)
    assert sst.rel_resid <= 1e-10 and hst.rel_resid <= 1e-10


@pytest.mark.parametrize("combo", COMBOS, ids=[f"np{a}_nq{b}_nw{c}" for a, b, c in COMBOS])
def test_curved_entry_points_accept_the_combination(combo):
    """The entry points built for the curved-wall mesh (velocity residual, P, C,
    tau_D, the div-div penalty, the inverse mass, the vorticity, the Neumann
    wall term) on every compiled combination."""
    npu, nq, nqw = combo
    cfg = MeshConfig(nx=2, ny=3, nz=2, wall_amp=0.3, k_u=npu - 1, nq_u=nq, nq_wn=nqw, k_p=npu - 2, nq_p=npu - 1,
                     nu=1.0 / 400)
    print(f"[gpu] curved coverage k_u={cfg.k_u} nq_u={nq} nq_wn={nqw}", flush=True)
    rng = np.random.default_rng(npu * 10 + nq + 1)
    mesh = Mesh(cfg, rng.uniform(0.5, 1.5, cfg.n_tau))
    u = torch.tensor(0.3 * rng.uniform(-1, 1, cfg.n_vel), device="cuda")
    p = torch.tensor(rng.uniform(-1, 1, cfg.n_p), device="cuda")
    td = mesh.divdiv_tau(u, 0.05)
    om = mesh.vorticity(u)
    outs = [mesh.apply_velocity_residual(u), mesh.apply_velocity_residual(u.float()), mesh.apply_pressure_gradient(p),
            mesh.apply_velocity_divergence(u), td, mesh.apply_divdiv(td, u), mesh.apply_inverse_mass(u), om,
            mesh.pressure_neumann([u], [om], (1.0,))]
    assert all(_finite(o) for o in outs)
