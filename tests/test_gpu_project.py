"""GPU switch-off rule of the enrichment and the cell-wise L2 projection onto
the refreshed enriched space (Sec. 3.2, eq. l2), against the CPU oracle,
through the C ABI.

Activity flags (an integer decided by floating point): bit-exact, on inputs
whose cells' largest y+ stays at least 1e-6 (relative) away from the
threshold.  Residuals: the 1e-12 bar of the velocity residual.  Projection:
||u_gpu - u_oracle||_inf <= PTOL ||u_old||_inf.  The oracle solves eq. l2 as a
weighted least-squares problem (SVD), the kernel by its closed form with
r = psi - P psi formed pointwise; both lose about eps sqrt(cond(M)) ~ 1e-13
relative when psi is close to a polynomial on the cell (cond(M) ~ 1e7 at the
y+ ranges used here), and the enrichment coefficient is divided by (r, r),
which amplifies that by up to another sqrt(cond(M)): PTOL = 1e-10.  Every
projected enriched cell is also held to the backward error of the normal
equation of eq. l2, ||M x_gpu - b|| <= 2 n eps (||M|| ||x_gpu|| + |Phi|^T W |u_old|)
per component, M = Phi^T W Phi and b = Phi^T W u_old from the oracle's basis
values: a bound that does not grow with cond(M).
"""
import numpy as np
import pytest
import torch

import oracle as O
from oracle import project as OP
from paper_1705_08813_amd import DgError, Mesh
from paper_1705_08813_amd.inputs import PRESETS, MeshConfig, Workload, draw_inputs
from numerics import EPS, backward_error

pytestmark = pytest.mark.gpu

PTOL = 1e-10

# wall-cell tops at y+ ~ 50-400 (the range where the enrichment is on)
CASES = {
    "k3": MeshConfig(nx=3, ny=3, nz=2, gamma=1.0, k_u=3, nq_u=5, nq_wn=8, nu=1.0 / 400),
    "k4": MeshConfig(nx=4, ny=4, nz=3, gamma=1.2, k_u=4, nq_u=7, nq_wn=8, nu=1.0 / 1000),
    "k5": MeshConfig(nx=2, ny=3, nz=2, gamma=0.8, k_u=5, nq_u=8, nq_wn=8, k_p=2, nq_p=3, nu=1.0 / 600),
    "k2": MeshConfig(nx=3, ny=4, nz=2, gamma=1.3, k_u=2, nq_u=4, nq_wn=8, k_p=1, nq_p=2, nu=1.0 / 800),
    "k4_lower_only": MeshConfig(nx=3, ny=3, nz=2, gamma=1.0, k_u=4, nq_u=7, nq_wn=8, nu=1.0 / 500, enrich_upper=0),
}


def _log(msg):
    print(msg, flush=True)


def _rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def _inputs(cfg, seed):
    return draw_inputs(Workload("p", cfg, seed, 0.5, 1.5))


def _nodes(cfg, seed, lo=0.4, hi=1.6):
    return np.random.default_rng(seed).uniform(lo, hi, (2, cfg.nz, cfg.nx))


def _max_yplus(cfg, tau=None, tau_nodes=None):
    """Largest y+ over the volume rule of every enriched cell (flat walls), in
    enriched-cell order, with numpy's Gauss rules."""
    g = 0.5 * (np.polynomial.legendre.leggauss(cfg.nq_wn)[0] + 1.0)
    gq = 0.5 * (np.polynomial.legendre.leggauss(cfg.nq_u)[0] + 1.0)
    eta = O.vertex_eta(cfg)
    out = []
    for e in O.enriched_cells(cfg):
        ex, ey, ez = e % cfg.nx, (e // cfg.nx) % cfg.ny, e // (cfg.nx * cfg.ny)
        w = 0 if ey == 0 else 1
        h = eta[ey + 1] - eta[ey]
        ytop = h * (g.max() if w == 0 else 1.0 - g.min())
        if tau_nodes is None:
            t = np.asarray(tau).reshape(2, cfg.nz, cfg.nx, cfg.nq_u, cfg.nq_u)[w, ez, ex].max()
        else:
            tn = np.asarray(tau_nodes).reshape(2, cfg.nz, cfg.nx)[w]
            jx, jz = (ex + 1) % cfg.nx, (ez + 1) % cfg.nz
            X, Z = np.meshgrid(gq, gq)
            t = ((1 - Z) * ((1 - X) * tn[ez, ex] + X * tn[ez, jx]) + Z * ((1 - X) * tn[jz, ex] + X * tn[jz, jx])).max()
        out.append(ytop * np.sqrt(t) / cfg.nu)
    return np.array(out)


def _threshold(*maxima):
    """A threshold between two distinct cell maxima (so that some cells are on
    and some off), at least 1e-6 relative away from every cell's value."""
    v = np.unique(np.concatenate(maxima))
    best = None
    for i in range(len(v) - 1):
        t = 0.5 * (v[i] + v[i + 1])
        gap = (v[i + 1] - v[i]) / t
        if gap > 2e-6 and (best is None or abs(i - len(v) // 2) < abs(best[1] - len(v) // 2)):
            best = (t, i)
    assert best is not None
    return float(best[0])


@pytest.mark.parametrize("name", ["k3", "k4", "k2"])
@pytest.mark.parametrize("nodal", [False, True])
def test_activity_flags_and_residual_match_oracle(name, nodal):
    base = CASES[name]
    inp = _inputs(base, 40)
    tn = _nodes(base, 41) if nodal else None
    mx = _max_yplus(base, tau=inp["tau"]) if not nodal else _max_yplus(base, tau_nodes=tn)
    cfg = base.with_(yplus_off=_threshold(mx))
    _log(f"[gpu] switch-off case={name} nodal={nodal} threshold={cfg.yplus_off:.3f}")
    mesh = Mesh(cfg, inp["tau"])
    if nodal:
        mesh.update_wall_shear_nodes(torch.tensor(tn, device="cuda"))
    flags = mesh.enrichment_active().cpu().numpy()
    ref = O.enrichment_active(cfg, tau=None if nodal else inp["tau"], tau_nodes=tn)
    assert np.array_equal(flags, ref)
    assert 0 < ref.sum() < ref.size
    r = mesh.apply_velocity_residual(torch.tensor(inp["u"], device="cuda")).cpu().numpy()
    ro = O.velocity_residual_nodal(cfg, inp["u"], tn) if nodal else O.velocity_residual(cfg, inp["u"], inp["tau"])
    n = cfg.ncell * 3 * (cfg.k_u + 1) ** 3
    assert _rel(r[:n], ro[:n]) <= 1e-12
    assert _rel(r[n:], ro[n:]) <= 1e-12
    off = np.repeat(ref == 0, 3)
    assert np.all(r[n:][off] == 0.0)


def _project_case(cfg, inp, tn_new=None, tau_new=None, tn_old=None):
    cells = O.enriched_cells(cfg)
    ps0 = O.psi_volume(cfg, cells, tau=None if tn_old is not None else inp["tau"], tau_nodes=tn_old)
    ps1 = O.psi_volume(cfg, cells, tau=tau_new, tau_nodes=tn_new)
    ref, cond = OP.project(cfg, inp["u"], ps0, ps1, return_cond=True)
    return ref, cond, ps0, ps1


def _check_backward(cfg, u_old, u_new, ps0, ps1, ks):
    """Backward error of eq. l2's normal equation in the enriched cells at positions ks."""
    n1 = (cfg.k_u + 1) ** 3
    off = cfg.ncell * 3 * n1
    cells = O.enriched_cells(cfg)
    worst = 0.0
    for k in ks:
        e = int(cells[k])
        A, b, babs = OP.l2_normal_equation(cfg, k, u_old, ps0[k], ps1[k])
        for c in range(3):
            rows = np.arange((e * 3 + c) * n1, (e * 3 + c + 1) * n1)
            if A.shape[0] == n1 + 1:
                rows = np.append(rows, off + 3 * k + c)
            eta = backward_error(A, u_new[rows], b[c], babs[c])
            worst = max(worst, eta / EPS)
            assert eta <= 2 * A.shape[0] * EPS, (k, c, eta / EPS)
    _log(f"[gpu]   worst backward error {worst:.1f} eps")


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("mode", ["per_point", "nodal", "switching"])
def test_projection_matches_oracle(name, mode):
    base = CASES[name]
    inp = _inputs(base, 50)
    tau1 = tn1 = tn0 = None
    if mode == "per_point":
        tau1 = np.random.default_rng(51).uniform(0.3, 2.0, base.n_tau)
        cfg = base
    elif mode == "nodal":
        tn1 = _nodes(base, 52)
        cfg = base
    else:
        # two nodal fields between which cells switch on and off
        tn0, tn1 = _nodes(base, 54, 0.2, 2.5), _nodes(base, 53, 0.2, 2.5)
        cfg = base.with_(yplus_off=_threshold(_max_yplus(base, tau_nodes=tn0), _max_yplus(base, tau_nodes=tn1)))
    _log(f"[gpu] projection case={name} mode={mode}")
    mesh = Mesh(cfg, inp["tau"])
    if tn0 is not None:
        mesh.update_wall_shear_nodes(torch.tensor(tn0, device="cuda"))
    if tau1 is not None:
        mesh.update_wall_shear(torch.tensor(tau1, device="cuda"))
    else:
        mesh.update_wall_shear_nodes(torch.tensor(tn1, device="cuda"))
    u = torch.tensor(inp["u"], device="cuda")
    un = mesh.project_velocity(u).cpu().numpy()
    ref, cond, ps0, ps1 = _project_case(cfg, inp, tn_new=tn1, tau_new=tau1, tn_old=tn0)
    err = _rel(un, ref)
    _log(f"[gpu]   max cond(M) {cond.max():.2e}  rel err {err:.2e}")
    assert err <= PTOL
    _check_backward(cfg, inp["u"], un, ps0, ps1, range(len(O.enriched_cells(cfg))))
    if mode == "switching":
        a0 = O.enrichment_active(cfg, tau_nodes=tn0)
        a1 = O.enrichment_active(cfg, tau_nodes=tn1)
        assert np.any(a0 != a1)
        if name in ("k3", "k4"):
            assert np.any((a0 == 1) & (a1 == 0)) and np.any((a0 == 0) & (a1 == 1))
        n = cfg.ncell * 3 * (cfg.k_u + 1) ** 3
        assert np.all(un[n:][np.repeat(a1 == 0, 3)] == 0.0)
    # cells without enrichment are copied bit for bit
    n3 = 3 * (cfg.k_u + 1) ** 3
    enr = set(O.enriched_cells(cfg).tolist())
    reg = np.array([e for e in range(cfg.ncell) if e not in enr])
    idx = (reg[:, None] * n3 + np.arange(n3)[None, :]).ravel()
    assert np.array_equal(un[idx], inp["u"][idx])


def test_projection_is_identity_before_any_update():
    cfg = CASES["k4"]
    inp = _inputs(cfg, 60)
    mesh = Mesh(cfg, inp["tau"])
    u = torch.tensor(inp["u"], device="cuda")
    un = mesh.project_velocity(u).cpu().numpy()
    assert _rel(un, inp["u"]) <= 1e-12


def test_projection_uses_the_last_two_spaces():
    cfg = CASES["k3"]
    inp = _inputs(cfg, 61)
    tn1, tn2 = _nodes(cfg, 62), _nodes(cfg, 63)
    mesh = Mesh(cfg, inp["tau"])
    mesh.update_wall_shear_nodes(torch.tensor(tn1, device="cuda"))
    mesh.update_wall_shear_nodes(torch.tensor(tn2, device="cuda"))
    un = mesh.project_velocity(torch.tensor(inp["u"], device="cuda")).cpu().numpy()
    cells = O.enriched_cells(cfg)
    ref = OP.project(cfg, inp["u"], O.psi_volume(cfg, cells, tau_nodes=tn1), O.psi_volume(cfg, cells, tau_nodes=tn2))
    assert _rel(un, ref) <= PTOL


def test_large_mesh_projection_sampled():
    # the 64x32x32 k=4 mesh with tau_w scaled so that the wall cells reach y+ ~ 100
    wl = PRESETS["large"]
    cfg = wl.mesh
    _log("[gpu] projection large mesh")
    inp = draw_inputs(wl)
    tau0 = 1600.0 * inp["tau"]
    tn1 = 1600.0 * _nodes(cfg, 70, 0.5, 1.5)
    mesh = Mesh(cfg, tau0)
    mesh.update_wall_shear_nodes(torch.tensor(tn1, device="cuda"))
    un = mesh.project_velocity(torch.tensor(inp["u"], device="cuda")).cpu().numpy()
    cells = O.enriched_cells(cfg)
    pick = np.unique(np.concatenate([[0, cells.size - 1], np.random.default_rng(71).integers(0, cells.size, 22)]))
    ps0 = np.zeros((cells.size, cfg.nq_u * cfg.nq_wn * cfg.nq_u))
    ps1 = np.zeros_like(ps0)
    ps0[pick] = O.psi_volume(cfg, cells[pick], tau=tau0)
    ps1[pick] = O.psi_volume(cfg, cells[pick], tau_nodes=tn1)
    ref = OP.project(cfg, inp["u"], ps0, ps1, only=pick)
    n3 = 3 * (cfg.k_u + 1) ** 3
    off = cfg.ncell * n3
    idx = np.concatenate([np.arange(e * n3, (e + 1) * n3) for e in cells[pick]] +
                         [(off + 3 * pick[:, None] + np.arange(3)[None, :]).ravel()])
    assert _rel(un[idx], ref[idx]) <= PTOL * np.abs(inp["u"]).max() / max(np.abs(ref[idx]).max(), 1e-300)
    _check_backward(cfg, inp["u"], un, ps0, ps1, pick)


def test_projection_rejects_bad_arguments():
    cfg = CASES["k3"]
    mesh = Mesh(cfg)
    u = torch.zeros(mesh.n_vel, dtype=torch.float64, device="cuda")
    with pytest.raises(ValueError):
        mesh.project_velocity(u, torch.zeros(7, dtype=torch.float64, device="cuda"))
    curved = Mesh(MeshConfig(nx=4, ny=3, nz=2, wall_amp=0.3, k_u=3, nq_u=5, nq_wn=8, k_p=2, nq_p=3))
    uc = torch.zeros(curved.n_vel, dtype=torch.float64, device="cuda")
    with pytest.raises(DgError) as ei:
        curved.project_velocity(uc)
    assert ei.value.code == -6


def test_switch_off_on_curved_wall_matches_oracle():
    # per-point tau_w on the cosine lower wall (y_h from the wall-vertex distances)
    base = MeshConfig(nx=4, ny=3, nz=2, wall_amp=0.3, k_u=3, nq_u=5, nq_wn=8, k_p=2, nq_p=3)
    inp = _inputs(base, 80)
    best = None
    for thr in np.linspace(20.0, 200.0, 91):
        a = O.enrichment_active(base.with_(yplus_off=float(thr)), tau=inp["tau"])
        if 0 < a.sum() < a.size and (best is None or abs(a.mean() - 0.5) < abs(best[1] - 0.5)):
            best = (float(thr), a.mean())
    assert best is not None
    cfg = base.with_(yplus_off=best[0])
    _log(f"[gpu] curved switch-off threshold={cfg.yplus_off:.1f}")
    mesh = Mesh(cfg, inp["tau"])
    flags = mesh.enrichment_active().cpu().numpy()
    assert np.array_equal(flags, O.enrichment_active(cfg, tau=inp["tau"]))
    r = mesh.apply_velocity_residual(torch.tensor(inp["u"], device="cuda")).cpu().numpy()
    ro = O.velocity_residual(cfg, inp["u"], inp["tau"])
    n = cfg.ncell * 3 * (cfg.k_u + 1) ** 3
    assert _rel(r[:n], ro[:n]) <= 1e-12 and _rel(r[n:], ro[n:]) <= 1e-12


def test_projection_in_place_equals_out_of_place():
    cfg = CASES["k4"]
    inp = _inputs(cfg, 90)
    mesh = Mesh(cfg, inp["tau"])
    mesh.update_wall_shear_nodes(torch.tensor(_nodes(cfg, 91), device="cuda"))
    u = torch.tensor(inp["u"], device="cuda")
    un = mesh.project_velocity(u)
    v = u.clone()
    mesh.project_velocity(v, v)
    torch.cuda.synchronize()
    assert torch.equal(un, v)
