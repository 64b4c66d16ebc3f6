"""Host-side parts of the serving path: the seeded request stream and the
footprint used for admission (no GPU needed)."""
import numpy as np

from paper_1705_08813_amd.inputs import ServingConfig, serving_requests
from paper_1705_08813_amd.serving import footprint_bytes
from paper_1705_08813_amd import _lib


def test_request_stream_is_seeded_and_covers_the_sets():
    cfg = ServingConfig()
    a = serving_requests(cfg)
    b = serving_requests(cfg)
    assert [(q.arrival, q.workload) for q in a] == [(q.arrival, q.workload) for q in b]
    assert len(a) == 512
    arr = np.array([q.arrival for q in a])
    assert arr[0] == 0.0 and np.all(np.diff(arr) >= 0)
    # mean gap of the exponential stream, within 4 standard errors
    gaps = np.diff(arr)
    assert abs(gaps.mean() - cfg.mean_interarrival) <= 4 * cfg.mean_interarrival / np.sqrt(len(gaps))
    grids = {(q.workload.mesh.nx, q.workload.mesh.ny, q.workload.mesh.nz) for q in a}
    ks = {q.workload.mesh.k_u for q in a}
    nus = {q.workload.mesh.nu for q in a}
    assert grids == set(cfg.grids) and ks == set(cfg.degrees) and nus == set(cfg.viscosities)
    for q in a:
        m = q.workload.mesh
        assert m.k_p == m.k_u - 1 and m.nq_p == m.k_p + 1 and m.nq_u == (3 * m.k_u) // 2 + 1
    assert len({q.workload.seed for q in a}) == len(a)


def test_footprint_counts_every_resident_buffer():
    sp = _lib.SolveParams(rtol=1e-10, max_outer=10, max_inner=0, cheb_degree=5, mixed=1)
    for q in serving_requests(ServingConfig(n_requests=16)):
        m = q.workload.mesh
        fp = footprint_bytes(q.workload, sp)
        # at least the four FP64 vectors plus the solver's 9 FP64 + 9 FP32 work vectors
        assert fp >= 8 * (2 * m.n_vel + 2 * m.n_p) + (9 * 8 + 9 * 4) * m.n_p
        assert fp < 1 << 30


def test_serving_footprint_leaves_out_the_projection_step_tables():
    """Served instances only apply operators and solve, so their meshes are
    set up without the projection-step tables; the mesh workspace then shrinks
    by at least the enriched cells' coupling cache (9 (k+1)^3 + 6 doubles per
    enriched cell) and the per-layer spectral factors (2 n^2 + n doubles per
    distinct cell height, n = 3 (k+1)^3)."""
    import ctypes
    L = _lib.lib()
    for q in serving_requests(ServingConfig(n_requests=8)):
        m = q.workload.mesh
        full = _lib.check(L.dg_mesh_workspace_bytes(ctypes.byref(_lib.params_from(m))))
        lean = _lib.check(L.dg_mesh_workspace_bytes(ctypes.byref(_lib.params_from(m.with_(omit_step_tables=1)))))
        n = 3 * (m.k_u + 1) ** 3
        assert full - lean >= 8 * (m.n_enriched * (9 * (m.k_u + 1) ** 3 + 6) + 2 * n * n + n)
