"""Pins of the oracle's dual-splitting steps (Sec. 4.1 eqs. convstep,
poisson, visc; Sec. 4.2 eqs. convstepspat, poissonspat, helmholtzspat)."""
import numpy as np
import pytest

import oracle as O
from oracle import project as OP
from oracle import step as OS
from paper_1705_08813_amd.inputs import PRESETS, MeshConfig, draw_inputs


def rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def test_mass_apply_inverts_inverse_mass():
    """The forward mass matrix undoes the oracle's inverse (same blocks)."""
    wl = PRESETS["tiny"]
    cfg = wl.mesh
    inp = draw_inputs(wl)
    psi = O.psi_volume(cfg, O.enriched_cells(cfg), tau=inp["tau"])
    x = np.random.default_rng(3).uniform(-1, 1, cfg.n_vel)
    y = OP.mass_apply(cfg, x, psi)
    assert rel(OP.inverse_mass(cfg, y, psi), x) < 1e-8   # enriched blocks: cond up to ~1e6
    # partition of unity: the polynomial rows of M applied to a constant field
    # sum to the cell volume times the constant
    n3 = (cfg.k_u + 1) ** 3
    ones = np.zeros(cfg.n_vel)
    ones[:cfg.ncell * 3 * n3] = 1.0
    tot = OP.mass_apply(cfg, ones, psi)[:cfg.ncell * 3 * n3].sum()
    assert abs(tot - 3 * cfg.Lx * 2.0 * cfg.Lz) < 1e-12 * tot


def test_helmholtz_constant_field_periodic():
    """No walls, no enrichment: A annihilates a constant field (no gradients,
    no jumps), so the Helmholtz solution is the right-hand side itself."""
    cfg = MeshConfig(nx=3, ny=2, nz=2, gamma=0.0, k_u=2, nq_u=4, k_p=1, nq_p=2, fully_periodic=1)
    n3 = (cfg.k_u + 1) ** 3
    b = np.zeros(cfg.n_vel)
    for c, v in enumerate((0.7, -0.2, 1.3)):
        for e in range(cfg.ncell):
            b[(e * 3 + c) * n3:(e * 3 + c + 1) * n3] = v
    x, its = OS.helmholtz_solve(cfg, None, None, 50.0, b, x0=np.zeros(cfg.n_vel))
    assert rel(x, b) < 1e-12


@pytest.mark.parametrize("gamma", [30.0, 3000.0])
def test_helmholtz_solves_the_unscaled_equation(gamma):
    """The M^{-1}-scaled GMRES solution satisfies gamma M x + A x = gamma M b
    with the forward mass matrix, walls and enrichment included."""
    wl = PRESETS["tiny"]
    cfg = wl.mesh
    inp = draw_inputs(wl)
    rng = np.random.default_rng(17)
    b = rng.uniform(-1, 1, cfg.n_vel)
    u_nut = rng.uniform(-1, 1, cfg.n_vel)
    x, its = OS.helmholtz_solve(cfg, u_nut, inp["tau"], gamma, b)
    r = OS.helmholtz_residual(cfg, u_nut, inp["tau"], gamma, b, x)
    psi = O.psi_volume(cfg, O.enriched_cells(cfg), tau=inp["tau"])
    scale = gamma * np.abs(OP.mass_apply(cfg, b, psi)).max()
    assert np.abs(r).max() < 1e-10 * scale
    assert its > 1
