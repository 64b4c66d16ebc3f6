"""CPU-side checks of the C ABI library: it loads, exports every symbol that
include/dgwm.h declares, and rejects invalid parameters without touching a
GPU (dg_mesh_workspace_bytes only validates and sizes)."""
import ctypes
import os
import re

import pytest

from paper_1705_08813_amd import _lib
from paper_1705_08813_amd.inputs import PRESETS, MeshConfig

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    txt = open(os.path.join(ROOT, "include", "dgwm.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(dg_[a-z_0-9]+)\s*\(", txt)))


def test_header_and_binding_agree():
    assert declared_symbols() == sorted(_lib.exported_symbols())


def test_library_exports_every_declared_symbol():
    L = _lib.lib()
    for name in declared_symbols():
        assert hasattr(L, name), name
    assert b"gfx950" in L.dg_build_info()


def ws_bytes(cfg):
    return _lib.lib().dg_mesh_workspace_bytes(ctypes.byref(_lib.params_from(cfg)))


def test_workspace_sizes_and_argument_errors():
    for name in ("tiny", "large", "precision", "curved"):
        assert ws_bytes(PRESETS[name].mesh) > 0
    good = PRESETS["tiny"].mesh
    bad = [good.with_(nx=0), good.with_(ny=1), good.with_(k_u=0), good.with_(nu=-1.0), good.with_(nq_u=40),
           good.with_(ip_factor_u=0.0), good.with_(gamma=float("nan")), good.with_(yplus_off=-1.0),
           good.with_(yplus_off=float("inf"))]
    for cfg in bad:
        assert ws_bytes(cfg) == -1, cfg
    assert ws_bytes(good.with_(k_u=6, nq_u=3)) == -6  # combination not compiled
    assert _lib.lib().dg_mesh_workspace_bytes(None) == -1
    assert b"NULL" in _lib.lib().dg_last_error()


def test_null_handles_are_rejected():
    L = _lib.lib()
    assert L.dg_num_dofs(None, 0) == -1
    assert L.dg_apply_velocity_residual(None, 0, None, None, None) == -1
    assert L.dg_apply_poisson(None, 0, None, None, None) == -1
    assert L.dg_poisson_diagonal(None, None, None) == -1
    assert L.dg_wall_shear_nodes(None, None, None, None) == -1
    assert L.dg_update_wall_shear_nodes(None, None, None) == -1
    assert L.dg_project_velocity(None, None, None, None) == -1
    assert L.dg_enrichment_active(None, None, None) == -1
    assert L.dg_apply_inverse_mass(None, None, None, None) == -1
    assert L.dg_apply_pressure_gradient(None, None, None, None) == -1
    assert L.dg_apply_velocity_divergence(None, None, None, None) == -1
    assert L.dg_divdiv_tau(None, None, 0.0, None, None) == -1
    assert L.dg_apply_divdiv(None, None, None, None, None) == -1
    assert L.dg_projection_step(None, None, None, None, 1.0, None, None) == -1


def test_large_workspace_fits_hbm():
    # mesh tables of the 64x32x32 k=4/k=3 case: far below one GPU's 288 GB
    n = ws_bytes(PRESETS["large"].mesh)
    assert 0 < n < 2 ** 30
