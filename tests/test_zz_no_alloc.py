"""The allocation-free Poisson solve (dg_solve_poisson_noalloc) against the
workspace solve (dg_solve_poisson), through the C ABI.

Both run the same kernels with the same launch shapes and fixed-order
reductions, so they must agree bit for bit; each result also meets the
binding solve check ||b' - A_oracle x|| <= 1.05e-10 ||b'||.  Two no-allocation
calls run back to back, the second on a smaller mesh, so the second reuses
the built-in array with the first call's contents still in it.
"""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1705_08813_amd import DgError, Mesh
from paper_1705_08813_amd.inputs import MeshConfig

pytestmark = pytest.mark.gpu

BIG = MeshConfig(nx=8, ny=8, nz=8, gamma=1.5, k_p=3, nq_p=4, k_u=2, nq_u=4)      # 32,768 unknowns, 4 levels
SMALL = MeshConfig(nx=4, ny=4, nz=6, gamma=1.0, k_p=2, nq_p=3, k_u=2, nq_u=4)    # 2,592 unknowns


def _relres(cfg, x, b):
    bp = b - b.mean()
    return float(np.linalg.norm(bp - O.poisson_apply(cfg, x)) / np.linalg.norm(bp))


@pytest.mark.parametrize("mixed", [True, False])
def test_noalloc_solve_equals_workspace_solve(mixed):
    print(f"[gpu] no-allocation solve mixed={mixed}", flush=True)
    cases = []
    for cfg, seed in ((BIG, 31), (SMALL, 32)):
        b = np.random.default_rng(seed).uniform(-1, 1, cfg.n_p)
        cases.append((cfg, b, Mesh(cfg), Mesh(cfg)))
    # two no-allocation calls in a row, the second on the smaller mesh
    got = []
    for cfg, b, m_na, _ in cases:
        sp = m_na.solve_params(mixed=mixed)
        x, st = m_na.solve_poisson_noalloc(torch.tensor(b, device="cuda"), sp=sp)
        got.append((x.cpu().numpy(), st.outer_its, st.rel_resid))
    for (cfg, b, _, m_ws), (x, its, rel) in zip(cases, got):
        sp = m_ws.solve_params(mixed=mixed)
        xr, st = m_ws.solve_poisson(torch.tensor(b, device="cuda"), sp=sp)
        xr = xr.cpu().numpy()
        print(f"[gpu]   n={cfg.n_p} its={its} rel={rel:.2e}", flush=True)
        assert its == st.outer_its and rel == st.rel_resid
        assert np.array_equal(x, xr)
        assert _relres(cfg, x, b) <= 1.05e-10


def test_noalloc_solve_repeats_on_one_mesh():
    # the same mesh twice in a row: the cached eigenvalue estimates and the
    # array's stale contents change nothing
    b = torch.tensor(np.random.default_rng(33).uniform(-1, 1, SMALL.n_p), device="cuda")
    mesh = Mesh(SMALL)
    x1, s1 = mesh.solve_poisson_noalloc(b)
    x1 = x1.clone()
    x2, s2 = mesh.solve_poisson_noalloc(b)
    torch.cuda.synchronize()
    assert torch.equal(x1, x2) and s1.outer_its == s2.outer_its


def test_noalloc_solve_rejects_a_mesh_beyond_the_array():
    # 32x32x16 cells at k_p = 3: 1,048,576 unknowns, about 110 MB of solve workspace
    cfg = MeshConfig(nx=32, ny=32, nz=16, gamma=1.5, k_p=3, nq_p=4, k_u=2, nq_u=4, enrich_lower=0, enrich_upper=0)
    mesh = Mesh(cfg)
    b = torch.zeros(cfg.n_p, dtype=torch.float64, device="cuda")
    with pytest.raises(DgError) as ei:
        mesh.solve_poisson_noalloc(b)
    assert ei.value.code == -2
