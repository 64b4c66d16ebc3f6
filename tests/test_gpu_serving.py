"""Serving path on the GPU: the batched velocity entry point against the
single-mesh one (bit-for-bit), the serving loop's results alone against in
a mix (bit-for-bit), one served request against the oracle, admission under
a device-memory budget, and failure isolation."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1705_08813_amd import Mesh, apply_velocity_residual_batched, batch_workspace
from paper_1705_08813_amd.inputs import MeshConfig, ServingConfig, Workload, draw_inputs, serving_requests
from paper_1705_08813_amd.serving import Server, footprint_bytes

pytestmark = pytest.mark.gpu


def _log(msg):
    print(msg, flush=True)


BATCH = [
    Workload("b0", MeshConfig(nx=4, ny=4, nz=4, k_u=3, nq_u=4, k_p=2, nq_p=3), 31, 1.0, 1.0),
    Workload("b1", MeshConfig(nx=3, ny=4, nz=2, gamma=1.3, k_u=2, nq_u=4, k_p=1, nq_p=2), 32, 0.5, 1.5),
    Workload("b2", MeshConfig(nx=5, ny=3, nz=3, gamma=1.8, k_u=4, nq_u=7), 33, 0.5, 1.5),
    Workload("b3", MeshConfig(nx=2, ny=4, nz=2, gamma=1.8, k_u=4, nq_u=7), 34, 0.5, 1.5),   # same group as b2
    Workload("b4", MeshConfig(nx=3, ny=3, nz=2, k_u=3, nq_u=5, fully_periodic=1), 35, 1.0, 1.0),
    Workload("b5", MeshConfig(nx=4, ny=3, nz=2, wall_amp=0.3, k_u=3, nq_u=5, k_p=2, nq_p=3), 36, 0.2, 2.0),
    Workload("b6", MeshConfig(nx=3, ny=3, nz=2, k_u=2, nq_u=4, nq_wn=4, k_p=1, nq_p=2, enrich_upper=0), 37, 0.5, 1.5),
]


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_batched_velocity_equals_single(dtype):
    _log(f"[gpu] batched velocity vs single dtype={dtype}")
    meshes, us = [], []
    for wl in BATCH:
        inp = draw_inputs(wl)
        meshes.append(Mesh(wl.mesh, inp["tau"]))
        us.append(torch.tensor(inp["u"], device="cuda", dtype=dtype))
    singles = [m.apply_velocity_residual(u) for m, u in zip(meshes, us)]
    rs = apply_velocity_residual_batched(meshes, us)
    # a second call with a smaller batch reuses the workspace
    ws = batch_workspace(len(meshes))
    rs2 = apply_velocity_residual_batched(meshes[2:5], us[2:5], workspace=ws)
    torch.cuda.synchronize()
    for i, (a, b) in enumerate(zip(singles, rs)):
        assert torch.equal(a, b), (BATCH[i].name, (a - b).abs().max().item())
    for a, b in zip(singles[2:5], rs2):
        assert torch.equal(a, b)


def test_batched_velocity_argument_errors():
    from paper_1705_08813_amd import DgError
    wl = BATCH[0]
    inp = draw_inputs(wl)
    m = Mesh(wl.mesh, inp["tau"])
    u = torch.tensor(inp["u"], device="cuda")
    r = torch.empty_like(u)
    with pytest.raises(DgError):          # two entries writing one output
        apply_velocity_residual_batched([m, m], [u, u], [r, r])
    with pytest.raises(ValueError):       # mixed precisions
        apply_velocity_residual_batched([m, m], [u, u.float()])
    small = torch.empty(64, dtype=torch.uint8, device="cuda")
    with pytest.raises(DgError):          # workspace too small
        apply_velocity_residual_batched([m], [u], workspace=small)


SMALL_STREAM = ServingConfig(n_requests=10, grids=((4, 4, 4), (8, 4, 4), (8, 8, 8)), applies=3, seed=7)


def _serve(reqs, **kw):
    srv = Server(keep_results=True, workers=4, applies=SMALL_STREAM.applies, **kw)
    return srv.run(reqs, time_scale=0.0)


def test_serving_alone_equals_mix():
    reqs = serving_requests(SMALL_STREAM)
    _log(f"[gpu] serving mix of {len(reqs)} requests")
    mix = _serve(reqs, slots=6)
    s = mix.summary()
    _log(f"[gpu]   {s}")
    assert s["completed"] == len(reqs)
    assert s["max_rel_resid"] <= 1e-10
    assert mix.peak_active <= 6
    for q in reqs[:4]:
        _log(f"[gpu]   alone rid={q.rid} {q.workload.mesh.nx}x{q.workload.mesh.ny}x{q.workload.mesh.nz} "
             f"k={q.workload.mesh.k_u}")
        alone = _serve([q], slots=1).outcomes[0]
        inmix = mix.outcomes[q.rid]
        assert alone.ok and inmix.ok
        assert torch.equal(alone.r, inmix.r)
        assert torch.equal(alone.x, inmix.x)
        # and the plain single-mesh call
        inp = draw_inputs(q.workload)
        m = Mesh(q.workload.mesh, inp["tau"])
        r1 = m.apply_velocity_residual(torch.tensor(inp["u"], device="cuda"))
        torch.cuda.synchronize()
        assert torch.equal(r1, inmix.r)


def test_served_request_matches_oracle():
    q = serving_requests(SMALL_STREAM)[0]
    cfg = q.workload.mesh
    _log(f"[gpu] served request vs oracle: {cfg.nx}x{cfg.ny}x{cfg.nz} k={cfg.k_u}")
    o = _serve([q], slots=1).outcomes[0]
    assert o.ok
    inp = draw_inputs(q.workload)
    r_orc = O.velocity_residual(cfg, inp["u"], inp["tau"])
    r = o.r.cpu().numpy()
    assert np.abs(r - r_orc).max() <= 1e-12 * np.abs(r_orc).max()
    b = inp["p"] - inp["p"].mean()
    x = o.x.cpu().numpy()
    assert np.linalg.norm(b - O.poisson_apply(cfg, x)) <= 1.05e-10 * np.linalg.norm(b)


def test_admission_respects_budget_and_slots():
    reqs = serving_requests(SMALL_STREAM)
    from paper_1705_08813_amd import _lib
    srv = Server(keep_results=False, workers=4, applies=SMALL_STREAM.applies, slots=3)
    fps = [footprint_bytes(q.workload, srv._sp()) for q in reqs]
    budget = 2 * max(fps)
    srv.budget = budget
    _log(f"[gpu] admission budget={budget} slots=3")
    rep = srv.run(reqs, time_scale=0.0)
    assert rep.summary()["completed"] == len(reqs)
    assert rep.peak_bytes <= budget
    assert rep.peak_active <= 3
    # a request larger than the whole budget is refused, the rest are served
    srv.budget = sorted(fps)[-1] - 1
    rep = srv.run(reqs, time_scale=0.0)
    big = [q.rid for q, f in zip(reqs, fps) if f > srv.budget]
    assert big
    for o in rep.outcomes:
        assert o.ok == (o.rid not in big)


def test_failed_solve_is_isolated():
    reqs = serving_requests(SMALL_STREAM)[:3]
    _log("[gpu] serving with an iteration cap that cannot converge")
    rep = Server(keep_results=False, workers=2, applies=1, solve_kw=dict(max_outer=1)).run(reqs, time_scale=0.0)
    assert len(rep.outcomes) == 3
    for o in rep.outcomes:
        assert not o.ok and "solve" in o.error
    # the server is still usable afterwards
    rep = Server(keep_results=False, workers=2, applies=1).run(reqs, time_scale=0.0)
    assert all(o.ok for o in rep.outcomes)
