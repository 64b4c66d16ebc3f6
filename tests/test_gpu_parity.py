"""GPU parity of the HIP operators against the FP64 CPU oracle, through the C ABI.

FP64: ||r_gpu - r_oracle||_inf <= 1e-12 ||r_oracle||_inf, checked separately
on the polynomial block and on the enrichment block of the velocity residual.
FP32: elementwise |r32 - r| <= c_m u32 R_abs + tiny, with R_abs the oracle
evaluated with absolute values of every factor (a bound on the magnitude of
every summand), u32 = 2^-24, and c_m = 4 (3 (nq + k + 1) + 40) covering the
longest accumulation chain of the sum-factorized evaluation (interpolation,
collocation derivative, transposed sweeps, six faces); inputs are the FP32
roundings, fed to the oracle as well.
"""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1705_08813_amd import Mesh
from paper_1705_08813_amd.inputs import PRESETS, MeshConfig, Workload, draw_inputs

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24


def _log(msg):
    print(msg, flush=True)


def _rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def _split(cfg, r):
    n = cfg.ncell * 3 * (cfg.k_u + 1) ** 3
    return r[:n], r[n:]


VEL_CASES = {
    "tiny": PRESETS["tiny"],
    "k2_stretched": Workload("k2", MeshConfig(nx=3, ny=4, nz=2, gamma=1.3, k_u=2, nq_u=4, k_p=1, nq_p=2), 11, 0.5, 1.5),
    "k4_large_like": Workload("k4", MeshConfig(nx=5, ny=4, nz=3, gamma=1.8, k_u=4, nq_u=7), 12, 0.5, 1.5),
    "k5_curved_rule": Workload("k5", MeshConfig(nx=2, ny=3, nz=2, gamma=0.7, k_u=5, nq_u=8, k_p=4, nq_p=5), 13, 0.2, 2.0),
    "k3_periodic": Workload("k3p", MeshConfig(nx=3, ny=3, nz=2, k_u=3, nq_u=5, nq_wn=8, fully_periodic=1), 14, 1, 1),
    "k4_lower_only": Workload("k4l", MeshConfig(nx=3, ny=3, nz=2, gamma=1.0, k_u=4, nq_u=7, enrich_upper=0), 15, 0.5, 1.5),
    "k3_nonsym": Workload("k3n", MeshConfig(nx=2, ny=3, nz=3, gamma=0.9, k_u=3, nq_u=5, theta=-1.0), 16, 0.5, 1.5),
    "k3_self_periodic": Workload("k3s", MeshConfig(nx=1, ny=2, nz=1, k_u=3, nq_u=4, nq_wn=8), 17, 0.5, 1.5),
    # curved lower wall y_w = -1 + 0.3 cos(2 pi x/Lx), isoparametric cells, both walls enriched
    "curved_k3": Workload("c3", MeshConfig(nx=4, ny=3, nz=2, wall_amp=0.3, k_u=3, nq_u=5, nq_wn=8, k_p=2, nq_p=3),
                          18, 0.2, 2.0),
    "curved_k5": Workload("c5", MeshConfig(nx=3, ny=3, nz=2, wall_amp=0.3, k_u=5, nq_u=8, nq_wn=8, k_p=4, nq_p=5),
                          19, 0.2, 2.0),
    "curved_k4_stretched": Workload("c4", MeshConfig(nx=3, ny=4, nz=2, gamma=1.2, wall_amp=0.25, k_u=4, nq_u=7,
                                                     nq_wn=8, enrich_upper=0), 20, 0.5, 1.5),
}


@pytest.mark.parametrize("name", list(VEL_CASES))
def test_velocity_residual_f64(name):
    wl = VEL_CASES[name]
    _log(f"[gpu] velocity f64 case={name}")
    inp = draw_inputs(wl)
    r_orc = O.velocity_residual(wl.mesh, inp["u"], inp["tau"])
    mesh = Mesh(wl.mesh, inp["tau"])
    r = mesh.apply_velocity_residual(torch.tensor(inp["u"], device="cuda"))
    torch.cuda.synchronize()
    r = r.cpu().numpy()
    rp, re = _split(wl.mesh, r)
    op, oe = _split(wl.mesh, r_orc)
    assert _rel(rp, op) <= 1e-12, _rel(rp, op)
    if oe.size:
        assert _rel(re, oe) <= 1e-12, _rel(re, oe)


@pytest.mark.parametrize("name", list(VEL_CASES))
def test_convective_f64(name):
    """dg_apply_convective against the oracle's convective form F^c (Sec. 4.2,
    eq. convstepspat), polynomial and enrichment blocks at 1e-12."""
    wl = VEL_CASES[name]
    _log(f"[gpu] convective f64 case={name}")
    inp = draw_inputs(wl)
    c_orc = O.convective_residual(wl.mesh, inp["u"], inp["tau"])
    mesh = Mesh(wl.mesh, inp["tau"])
    c = mesh.apply_convective(torch.tensor(inp["u"], device="cuda")).cpu().numpy()
    cp, ce = _split(wl.mesh, c)
    op, oe = _split(wl.mesh, c_orc)
    assert _rel(cp, op) <= 1e-12, _rel(cp, op)
    if oe.size:
        assert _rel(ce, oe) <= 1e-12, _rel(ce, oe)


@pytest.mark.parametrize("name", ["tiny", "k4_large_like", "k3_periodic", "curved_k3", "k5_curved_rule", "curved_k5",
                                  "curved_k4_stretched"])
def test_velocity_residual_f32_bound(name):
    wl = VEL_CASES[name]
    _log(f"[gpu] velocity f32 case={name}")
    inp = draw_inputs(wl)
    u32 = inp["u"].astype(np.float32)
    u_r = u32.astype(np.float64)
    r_orc = O.velocity_residual(wl.mesh, u_r, inp["tau"])
    r_abs = O.velocity_residual(wl.mesh, u_r, inp["tau"], absmode=True)
    mesh = Mesh(wl.mesh, inp["tau"])
    r = mesh.apply_velocity_residual(torch.tensor(u32, device="cuda")).cpu().numpy().astype(np.float64)
    m = 3 * (wl.mesh.nq_u + wl.mesh.k_u + 1) + 40
    bound = 4 * m * U32 * r_abs + 1e-30
    err = np.abs(r - r_orc)
    worst = float((err / bound).max())
    _log(f"[gpu]   max rel err {_rel(r, r_orc):.3e}, max err/bound {worst:.3f}")
    assert worst <= 1.0


POI_CASES = {
    "tiny": PRESETS["tiny"].mesh,
    "k1": MeshConfig(nx=3, ny=4, nz=2, gamma=1.3, k_p=1, nq_p=2),
    "k3_stretched": MeshConfig(nx=4, ny=5, nz=3, gamma=1.8, k_p=3, nq_p=4),
    "k4": MeshConfig(nx=2, ny=3, nz=2, gamma=0.5, k_p=4, nq_p=5, k_u=5, nq_u=8),
    "k5": MeshConfig(nx=2, ny=2, nz=2, k_p=5, nq_p=6, k_u=5, nq_u=8),
    "k2_periodic": MeshConfig(nx=3, ny=3, nz=3, k_p=2, nq_p=3, k_u=3, nq_u=5, fully_periodic=1),
    "k3_self_periodic": MeshConfig(nx=1, ny=3, nz=1, gamma=1.0, k_p=3, nq_p=4, k_u=3, nq_u=4, nq_wn=8),
}


@pytest.mark.parametrize("name", list(POI_CASES))
def test_poisson_f64_and_diagonal(name):
    cfg = POI_CASES[name]
    _log(f"[gpu] poisson f64 case={name}")
    p = np.random.default_rng(21).uniform(-1, 1, cfg.n_p)
    y_orc = O.poisson_apply(cfg, p)
    mesh = Mesh(cfg)
    y = mesh.apply_poisson(torch.tensor(p, device="cuda"))
    d = mesh.poisson_diagonal()
    torch.cuda.synchronize()
    assert _rel(y.cpu().numpy(), y_orc) <= 1e-12
    assert _rel(d.cpu().numpy(), O.poisson_diag(cfg)) <= 1e-12


@pytest.mark.parametrize("name", ["tiny", "k3_stretched", "k2_periodic"])
def test_poisson_f32_bound(name):
    cfg = POI_CASES[name]
    _log(f"[gpu] poisson f32 case={name}")
    p32 = np.random.default_rng(22).uniform(-1, 1, cfg.n_p).astype(np.float32)
    pr = p32.astype(np.float64)
    y_orc = O.poisson_apply(cfg, pr)
    y_abs = O.poisson_apply(cfg, pr, absmode=True)
    mesh = Mesh(cfg)
    y = mesh.apply_poisson(torch.tensor(p32, device="cuda")).cpu().numpy().astype(np.float64)
    m = 3 * (cfg.nq_p + cfg.k_p + 1) + 40
    worst = float((np.abs(y - y_orc) / (4 * m * U32 * y_abs + 1e-30)).max())
    _log(f"[gpu]   max rel err {_rel(y, y_orc):.3e}, max err/bound {worst:.3f}")
    assert worst <= 1.0


def _enrichment_rows(m, cells):
    n3 = (m.k_u + 1) ** 3
    off = m.ncell * 3 * n3
    rows = []
    for e in cells:
        ex, ey, ez = e % m.nx, (e // m.nx) % m.ny, e // (m.nx * m.ny)
        if ey in (0, m.ny - 1):
            k = ex + m.nx * ((0 if ey == 0 else 1) + 2 * ez)
            rows += [off + 3 * k + c for c in range(3)]
    return np.array(rows, dtype=np.int64)


def test_large_config_full_field():
    """64x32x32, tanh 1.8, k=4 / k=3, in the configuration the benchmark times:
    the whole Poisson output and the whole velocity residual (polynomial and
    enrichment blocks) against the oracle."""
    wl = PRESETS["large"]
    m = wl.mesh
    _log("[gpu] large config: setup")
    inp = draw_inputs(wl)
    mesh = Mesh(m, inp["tau"])
    _log("[gpu] large config: poisson f64")
    y = mesh.apply_poisson(torch.tensor(inp["p"], device="cuda"))
    torch.cuda.synchronize()
    assert _rel(y.cpu().numpy(), O.poisson_apply(m, inp["p"])) <= 1e-12
    _log("[gpu] large config: velocity f64, oracle on every cell")
    r = mesh.apply_velocity_residual(torch.tensor(inp["u"], device="cuda")).cpu().numpy()
    r_orc = O.velocity_residual(m, inp["u"], inp["tau"])
    rp, re = _split(m, r)
    op, oe = _split(m, r_orc)
    _log(f"[gpu]   rel poly {_rel(rp, op):.2e} enr {_rel(re, oe):.2e}")
    assert _rel(rp, op) <= 1e-12 and _rel(re, oe) <= 1e-12


def test_repeat_applies_are_bitwise_identical():
    """Deterministic: no atomics, fixed reduction order."""
    wl = PRESETS["tiny"]
    inp = draw_inputs(wl)
    mesh = Mesh(wl.mesh, inp["tau"])
    u = torch.tensor(inp["u"], device="cuda")
    p = torch.tensor(inp["p"], device="cuda")
    r1 = mesh.apply_velocity_residual(u).clone()
    r2 = mesh.apply_velocity_residual(u)
    y1 = mesh.apply_poisson(p).clone()
    y2 = mesh.apply_poisson(p)
    torch.cuda.synchronize()
    assert torch.equal(r1, r2) and torch.equal(y1, y2)


def test_wall_shear_update_matches_fresh_setup():
    wl = VEL_CASES["k4_lower_only"]
    inp = draw_inputs(wl)
    tau2 = np.random.default_rng(99).uniform(0.3, 2.0, wl.mesh.n_tau)
    mesh = Mesh(wl.mesh, inp["tau"])
    mesh.update_wall_shear(torch.tensor(tau2, device="cuda"))
    u = torch.tensor(inp["u"], device="cuda")
    r = mesh.apply_velocity_residual(u).cpu().numpy()
    r_orc = O.velocity_residual(wl.mesh, inp["u"], tau2)
    assert _rel(r, r_orc) <= 1e-12


def test_curved_config_full_field():
    """48x24x24 curved channel, k=5 (8 Gauss points), both walls enriched,
    tau_w ~ U[0.2, 2]: every cell against the oracle, FP64."""
    wl = PRESETS["curved"]
    m = wl.mesh
    _log("[gpu] curved config: setup")
    inp = draw_inputs(wl, want=("u", "tau"))
    mesh = Mesh(m, inp["tau"])
    r = mesh.apply_velocity_residual(torch.tensor(inp["u"], device="cuda")).cpu().numpy()
    _log("[gpu] curved config: oracle on every cell")
    r_orc = O.velocity_residual(m, inp["u"], inp["tau"])
    rp, re = _split(m, r)
    op, oe = _split(m, r_orc)
    _log(f"[gpu]   rel poly {_rel(rp, op):.2e} enr {_rel(re, oe):.2e}")
    assert _rel(rp, op) <= 1e-12 and _rel(re, oe) <= 1e-12


def test_curved_config_f32_bound_sampled():
    """The FP32 apply the benchmark times on the 48x24x24 curved k=5 mesh:
    sampled cells (both enriched layers, their neighbours, interior) against
    the elementwise bound 4 m u32 R_abs, the oracle run on the FP32 roundings."""
    wl = PRESETS["curved"]
    m = wl.mesh
    _log("[gpu] curved config f32: setup")
    inp = draw_inputs(wl, want=("u", "tau"))
    u32 = inp["u"].astype(np.float32)
    u_r = u32.astype(np.float64)
    mesh = Mesh(m, inp["tau"])
    r = mesh.apply_velocity_residual(torch.tensor(u32, device="cuda")).cpu().numpy().astype(np.float64)
    rng = np.random.default_rng(9)
    cells = set(rng.integers(0, m.ncell, 60).tolist())
    for ey in (0, 1, m.ny - 2, m.ny - 1):
        for _ in range(15):
            cells.add(int(rng.integers(0, m.nx)) + m.nx * (ey + m.ny * int(rng.integers(0, m.nz))))
    cells = np.array(sorted(cells), dtype=np.int64)
    _log(f"[gpu] curved config f32: oracle on {cells.size} cells")
    r_orc = O.velocity_residual(m, u_r, inp["tau"], cells=cells)
    r_abs = O.velocity_residual(m, u_r, inp["tau"], cells=cells, absmode=True)
    n3 = (m.k_u + 1) ** 3
    rows = np.concatenate([(cells[:, None] * 3 * n3 + np.arange(3 * n3)[None, :]).ravel(),
                           _enrichment_rows(m, cells)])
    mq = 3 * (m.nq_u + m.k_u + 1) + 40
    worst = float((np.abs(r[rows] - r_orc[rows]) / (4 * mq * U32 * r_abs[rows] + 1e-30)).max())
    _log(f"[gpu]   max rel err {_rel(r[rows], r_orc[rows]):.3e}, max err/bound {worst:.3f}")
    assert worst <= 1.0


# van Driest's enrichment (Sec. 3.2, eq. psi; Appendix A evaluation on the GPU,
# composite Gauss from zero in the oracle).  The meshes span wall-cell y+ from
# below the first support point to the 361..946 slice.
VD_CASES = {
    "vd_tiny": Workload("vd0", MeshConfig(nx=4, ny=4, nz=4, k_u=3, nq_u=4, k_p=2, nq_p=3, psi_kind=1), 41, 1.0, 1.0),
    "vd_k4_stretched": Workload("vd1", MeshConfig(nx=3, ny=4, nz=2, gamma=1.8, k_u=4, nq_u=7, psi_kind=1), 42,
                                0.5, 1.5),
    "vd_k3_high_re": Workload("vd2", MeshConfig(nx=3, ny=3, nz=2, k_u=3, nq_u=5, psi_kind=1, nu=1.0 / 2000.0), 43,
                              0.5, 2.0),
    "vd_curved_k3": Workload("vd3", MeshConfig(nx=4, ny=3, nz=2, wall_amp=0.3, k_u=3, nq_u=5, k_p=2, nq_p=3,
                                               psi_kind=1), 44, 0.2, 2.0),
}


@pytest.mark.parametrize("name", list(VD_CASES))
def test_velocity_residual_vandriest_f64(name):
    wl = VD_CASES[name]
    _log(f"[gpu] velocity f64 van Driest case={name}")
    inp = draw_inputs(wl)
    r_orc = O.velocity_residual(wl.mesh, inp["u"], inp["tau"])
    mesh = Mesh(wl.mesh, inp["tau"])
    r = mesh.apply_velocity_residual(torch.tensor(inp["u"], device="cuda"))
    torch.cuda.synchronize()
    rp, re = _split(wl.mesh, r.cpu().numpy())
    op, oe = _split(wl.mesh, r_orc)
    _log(f"[gpu]   rel poly {_rel(rp, op):.2e} enr {_rel(re, oe):.2e}")
    assert _rel(rp, op) <= 1e-12, _rel(rp, op)
    assert _rel(re, oe) <= 1e-12, _rel(re, oe)
