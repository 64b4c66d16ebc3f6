"""Steps of the dual-splitting scheme (arXiv 1705.08813, Sec. 4.1 eqs.
convstep, poisson, bc_d_pres, visc; Sec. 4.2 eqs. convstepspat, poissonspat,
projectionspat, helmholtzspat), composed from the oracle's operators.

TEST INFRASTRUCTURE ONLY (never used by the product).

Library solvers serve as the solution steps: SciPy's GMRES for the
Helmholtz equation, NumPy's dense least squares for the singular pressure
equation on small meshes.  Flat (box) meshes only.
"""
from __future__ import annotations

import numpy as np

from . import enriched_cells, psi_volume, viscous_multiscale
from .project import inverse_mass, mass_apply


def _psi(cfg, tau):
    cells = enriched_cells(cfg)
    return psi_volume(cfg, cells, tau=tau) if cells.size else np.zeros((0, 1))


def helmholtz_solve(cfg, u_nut, tau, gamma, b, rtol=1e-11, x0=None):
    """x with gamma M x + A x = gamma M b (Sec. 4.2 eq. helmholtzspat,
    gamma = gamma0/dt, A = -F^nu of eq. viscous_multiscale with nu_t from
    the enrichment of u_nut), by GMRES on the M^{-1}-scaled form
    gamma x + M^{-1} A x = gamma b.  Returns (x, GMRES iterations)."""
    import scipy.sparse.linalg as sla
    psi = _psi(cfg, tau)
    n = cfg.n_vel
    u_nut = np.zeros(n) if u_nut is None else np.asarray(u_nut, dtype=np.float64)   # nu_t stays fixed

    def H(x):
        return gamma * x + inverse_mass(cfg, viscous_multiscale(cfg, x, u_nut=u_nut, tau=tau), psi)

    op = sla.LinearOperator((n, n), matvec=H, dtype=np.float64)
    its = [0]

    def cb(_):
        its[0] += 1

    x, info = sla.gmres(op, gamma * np.asarray(b, dtype=np.float64), x0=b if x0 is None else x0, rtol=rtol, atol=0.0,
                        restart=150, maxiter=8, callback=cb, callback_type="pr_norm")
    if info != 0:
        raise RuntimeError(f"oracle GMRES did not converge: {info}")
    return x, its[0]


def helmholtz_residual(cfg, u_nut, tau, gamma, b, x):
    """gamma M x + A x - gamma M b with the forward mass matrix (no inverse)."""
    psi = _psi(cfg, tau)
    u_nut = np.zeros(cfg.n_vel) if u_nut is None else u_nut
    return gamma * mass_apply(cfg, x, psi) + viscous_multiscale(cfg, x, u_nut=u_nut, tau=tau) \
        - gamma * mass_apply(cfg, b, psi)
