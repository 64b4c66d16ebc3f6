"""Seeded synthetic inputs and named workload presets.

This module is shared by the test suite, the benchmark and the smoke check to
feed the *same* numbers to the HIP library and to the CPU oracle.  It holds no
arithmetic of the method: only preset sizes and random draws of the right
shapes.

Workloads stand in for the paper's turbulent-channel runs (Sec. 5.1: box
2pi x 2 x pi, tanh wall-normal grading, polynomial degree k around 4, one
enriched wall layer) and for its curved-wall periodic-hill runs (Sec. 5.2),
with coefficients drawn uniformly instead of taken from a turbulent flow.

Draw order per preset (one ``numpy.random.default_rng(seed)`` stream):
polynomial velocity DoFs, enrichment DoFs, wall shear stress, then the
pressure vector / right-hand side.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, asdict, replace

import numpy as np


@dataclass(frozen=True)
class MeshConfig:
    """Plain numbers describing one channel instance (no derived quantities)."""

    nx: int
    ny: int
    nz: int
    Lx: float = 2.0 * math.pi
    Lz: float = math.pi
    gamma: float = 0.0
    wall_amp: float = 0.0
    k_u: int = 4
    k_p: int = 3
    nq_u: int = 7
    nq_p: int = 4
    nq_wn: int = 8
    enrich_lower: int = 1
    enrich_upper: int = 1
    fully_periodic: int = 0
    nu: float = 1.0 / 180.0
    kappa: float = 0.41
    B: float = 5.17
    ip_factor_u: float = 1.0
    ip_factor_p: float = 1.0
    wall_ip_mult: float = 10.0
    theta: float = 1.0
    psi_kind: int = 0          # 0: Spalding's law, 1: van Driest's law
    A_plus: float = 26.0
    yplus_off: float = 0.0     # > 0: switch a wall cell's enrichment off while all its points have y+ below this
    enrich_degree: int = 0     # tensor degree l of the enrichment weights (0: 3, 1: 24 DoFs per enriched cell)
    omit_step_tables: int = 0  # 1: no projection-step tables in the mesh workspace (operators and solves only)

    def as_dict(self):
        return asdict(self)

    def with_(self, **kw):
        return replace(self, **kw)

    # ---- layout counts (shapes only) ----
    @property
    def ncell(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def n_enriched(self) -> int:
        if self.fully_periodic:
            return 0
        layers = 0
        if self.enrich_lower:
            layers += 1
        if self.enrich_upper and (self.ny > 1 or not self.enrich_lower):
            layers += 1
        return self.nx * self.nz * layers

    @property
    def n_vel(self) -> int:
        return self.ncell * 3 * (self.k_u + 1) ** 3 + self.n_enr_dofs

    @property
    def n_enr_dofs(self) -> int:
        """Enrichment unknowns: 3 (l+1)^3 per enriched cell."""
        return 3 * (self.enrich_degree + 1) ** 3 * self.n_enriched

    @property
    def n_p(self) -> int:
        return self.ncell * (self.k_p + 1) ** 3

    @property
    def n_tau(self) -> int:
        return 2 * self.nz * self.nx * self.nq_u * self.nq_u


@dataclass(frozen=True)
class Workload:
    name: str
    mesh: MeshConfig
    seed: int
    tau_lo: float
    tau_hi: float
    note: str = ""


PRESETS = {
    # 4x4x4 uniform box, k=3 (4^3 Gauss points, 8 wall-normal in enriched
    # cells), pressure k=2, tau_w = 1.
    "tiny": Workload("tiny", MeshConfig(nx=4, ny=4, nz=4, gamma=0.0, k_u=3, k_p=2, nq_u=4, nq_p=3, nq_wn=8),
                     seed=1, tau_lo=1.0, tau_hi=1.0),
    # 64x32x32, tanh grading 1.8, k=4 velocity (floor(3k/2)+1 = 7 points),
    # k=3 pressure (k+1 = 4 points), tau_w ~ U[0.5, 1.5].
    "large": Workload("large", MeshConfig(nx=64, ny=32, nz=32, gamma=1.8, k_u=4, k_p=3, nq_u=7, nq_p=4, nq_wn=8),
                      seed=2, tau_lo=0.5, tau_hi=1.5),
    # same mesh, Poisson k=3 solve
    "precision": Workload("precision", MeshConfig(nx=64, ny=32, nz=32, gamma=1.8, k_u=4, k_p=3, nq_u=7, nq_p=4,
                                                  nq_wn=8), seed=3, tau_lo=0.5, tau_hi=1.5),
    # 48x24x24 with a cosine lower wall, k=5 velocity (8 points), both walls
    # enriched, tau_w ~ U[0.2, 2.0].
    "curved": Workload("curved", MeshConfig(nx=48, ny=24, nz=24, gamma=0.0, wall_amp=0.3, k_u=5, k_p=4, nq_u=8,
                                            nq_p=5, nq_wn=8), seed=4, tau_lo=0.2, tau_hi=2.0),
}


def default_nq_u(k: int) -> int:
    """Gauss points per direction for nonlinear terms: floor(3k/2)+1."""
    return (3 * k) // 2 + 1


def draw_inputs(wl: Workload, want=("u", "tau", "p"), dtype=np.float64):
    """Draw the preset's inputs in the fixed order u_poly, u_enr, tau, p."""
    m = wl.mesh
    rng = np.random.default_rng(wl.seed)
    out = {}
    npu3 = (m.k_u + 1) ** 3
    u_poly = rng.uniform(-1.0, 1.0, size=m.ncell * 3 * npu3)
    u_enr = rng.uniform(-1.0, 1.0, size=m.n_enr_dofs)
    if wl.tau_lo == wl.tau_hi:
        tau = np.full(m.n_tau, wl.tau_lo)
    else:
        tau = rng.uniform(wl.tau_lo, wl.tau_hi, size=m.n_tau)
    p = rng.uniform(-1.0, 1.0, size=m.n_p)
    if "u" in want:
        out["u"] = np.concatenate([u_poly, u_enr]).astype(dtype)
    if "tau" in want:
        out["tau"] = tau
    if "p" in want:
        out["p"] = p.astype(dtype)
    return out


def random_vector(n: int, seed: int, lo=-1.0, hi=1.0):
    return np.random.default_rng(seed).uniform(lo, hi, size=n)


# ---------------------------------------------------------------- serving ---

@dataclass(frozen=True)
class ServingConfig:
    """A seeded stream of channel-instance requests (Poisson arrivals)."""

    n_requests: int = 512
    mean_interarrival: float = 0.005          # seconds (200 requests/s)
    seed: int = 5
    grids: tuple = ((8, 8, 8), (16, 8, 8), (16, 16, 16), (32, 16, 16))
    degrees: tuple = (2, 3, 4, 5)
    viscosities: tuple = (1.0 / 180.0, 1.0 / 395.0, 1.0 / 590.0)
    gamma: float = 1.8
    tau_lo: float = 0.5
    tau_hi: float = 1.5
    applies: int = 10                         # velocity-residual applies per request

    def with_(self, **kw):
        return replace(self, **kw)


@dataclass(frozen=True)
class Request:
    rid: int
    arrival: float                            # seconds after the stream starts
    workload: Workload


def serving_requests(cfg: ServingConfig):
    """Arrival times (exponential gaps), then per request the grid, degree
    and viscosity drawn uniformly from the listed sets.  Pressure degree is
    k - 1 with k_p + 1 Gauss points; velocity uses floor(3k/2)+1 points."""
    rng = np.random.default_rng(cfg.seed)
    gaps = rng.exponential(cfg.mean_interarrival, size=cfg.n_requests)
    arrivals = np.cumsum(gaps) - gaps[0]
    gi = rng.integers(0, len(cfg.grids), size=cfg.n_requests)
    ki = rng.integers(0, len(cfg.degrees), size=cfg.n_requests)
    vi = rng.integers(0, len(cfg.viscosities), size=cfg.n_requests)
    out = []
    for i in range(cfg.n_requests):
        nx, ny, nz = cfg.grids[gi[i]]
        k = int(cfg.degrees[ki[i]])
        mesh = MeshConfig(nx=nx, ny=ny, nz=nz, gamma=cfg.gamma, k_u=k, k_p=k - 1, nq_u=default_nq_u(k),
                          nq_p=k, nq_wn=8, nu=float(cfg.viscosities[vi[i]]))
        wl = Workload(f"request{i}", mesh, seed=cfg.seed * 1_000_003 + i, tau_lo=cfg.tau_lo, tau_hi=cfg.tau_hi)
        out.append(Request(i, float(arrivals[i]), wl))
    return out
