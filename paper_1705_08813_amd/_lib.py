"""ctypes binding of libdgwm.so (the C ABI in include/dgwm.h).

Argument marshalling only: every step of the computation runs in the HIP
library.  torch supplies device memory and streams.  If the shared library
is missing, importing the binding raises instead of falling back to anything.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdgwm.so")

DG_F64, DG_F32 = 0, 1
ERRORS = {-1: "DG_ERR_ARG", -2: "DG_ERR_WORKSPACE", -3: "DG_ERR_HIP", -4: "DG_ERR_NONFINITE",
          -5: "DG_ERR_NOT_CONVERGED", -6: "DG_ERR_UNSUPPORTED"}


class DgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class MeshParams(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("Lx", ctypes.c_double), ("Lz", ctypes.c_double),
        ("gamma", ctypes.c_double), ("wall_amp", ctypes.c_double),
        ("k_u", ctypes.c_int32), ("k_p", ctypes.c_int32),
        ("nq_u", ctypes.c_int32), ("nq_p", ctypes.c_int32), ("nq_wn", ctypes.c_int32),
        ("enrich_lower", ctypes.c_int32), ("enrich_upper", ctypes.c_int32), ("fully_periodic", ctypes.c_int32),
        ("nu", ctypes.c_double), ("kappa", ctypes.c_double), ("B", ctypes.c_double),
        ("ip_factor_u", ctypes.c_double), ("ip_factor_p", ctypes.c_double),
        ("wall_ip_mult", ctypes.c_double), ("theta", ctypes.c_double),
        ("psi_kind", ctypes.c_int32), ("A_plus", ctypes.c_double), ("yplus_off", ctypes.c_double),
        ("enrich_degree", ctypes.c_int32), ("omit_step_tables", ctypes.c_int32),
    ]


class SolveParams(ctypes.Structure):
    _fields_ = [("rtol", ctypes.c_double), ("max_outer", ctypes.c_int32), ("max_inner", ctypes.c_int32),
                ("cheb_degree", ctypes.c_int32), ("mixed", ctypes.c_int32),
                ("multigrid", ctypes.c_int32), ("coarse_degree", ctypes.c_int32)]


class GmresParams(ctypes.Structure):
    _fields_ = [("rtol", ctypes.c_double), ("max_iter", ctypes.c_int32), ("restart", ctypes.c_int32)]


class GmresStats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("restarts", ctypes.c_int32), ("rel_resid", ctypes.c_double),
                ("seconds", ctypes.c_double)]


class SolveStats(ctypes.Structure):
    _fields_ = [("outer_its", ctypes.c_int32), ("inner_its_total", ctypes.c_int32),
                ("op_applies_f64", ctypes.c_int32), ("op_applies_f32", ctypes.c_int32),
                ("rel_resid", ctypes.c_double), ("seconds", ctypes.c_double)]


class StepParams(ctypes.Structure):
    _fields_ = [("dt", ctypes.c_double), ("gamma0", ctypes.c_double), ("alpha", ctypes.c_double * 2),
                ("beta", ctypes.c_double * 2), ("order", ctypes.c_int32), ("f", ctypes.c_double * 3),
                ("dt_over_cr", ctypes.c_double), ("c_des", ctypes.c_double), ("beta_des", ctypes.c_double),
                ("poisson", SolveParams), ("helmholtz", GmresParams)]


class StepStats(ctypes.Structure):
    _fields_ = [("poisson", SolveStats), ("helmholtz", GmresStats), ("seconds", ctypes.c_double),
                ("projection_its", ctypes.c_int32)]


# every symbol include/dgwm.h declares, with its signature
_VP = ctypes.c_void_p
_SIGS = {
    "dg_mesh_workspace_bytes": (ctypes.c_int64, [ctypes.POINTER(MeshParams)]),
    "dg_setup_mesh": (ctypes.c_int, [ctypes.POINTER(MeshParams), ctypes.POINTER(ctypes.c_double), _VP,
                                     ctypes.c_size_t, _VP, ctypes.POINTER(_VP)]),
    "dg_update_wall_shear": (ctypes.c_int, [_VP, _VP, _VP]),
    "dg_wall_shear_nodes": (ctypes.c_int, [_VP, _VP, _VP, _VP]),
    "dg_update_wall_shear_nodes": (ctypes.c_int, [_VP, _VP, _VP]),
    "dg_project_velocity": (ctypes.c_int, [_VP, _VP, _VP, _VP]),
    "dg_apply_inverse_mass": (ctypes.c_int, [_VP, _VP, _VP, _VP]),
    "dg_apply_pressure_gradient": (ctypes.c_int, [_VP, _VP, _VP, _VP]),
    "dg_apply_velocity_divergence": (ctypes.c_int, [_VP, _VP, _VP, _VP]),
    "dg_divdiv_tau": (ctypes.c_int, [_VP, _VP, ctypes.c_double, _VP, _VP]),
    "dg_apply_divdiv": (ctypes.c_int, [_VP, _VP, _VP, _VP, _VP]),
    "dg_projection_step": (ctypes.c_int, [_VP, _VP, _VP, _VP, ctypes.c_double, _VP, _VP]),
    "dg_enrichment_active": (ctypes.c_int, [_VP, _VP, _VP]),
    "dg_eddy_viscosity_points": (ctypes.c_int64, [_VP]),
    "dg_eddy_viscosity": (ctypes.c_int, [_VP, _VP, ctypes.c_double, ctypes.c_double, _VP, _VP]),
    "dg_apply_viscous_multiscale": (ctypes.c_int, [_VP, _VP, _VP, _VP, _VP]),
    "dg_num_dofs": (ctypes.c_int64, [_VP, ctypes.c_int]),
    "dg_num_enriched": (ctypes.c_int64, [_VP]),
    "dg_destroy_mesh": (None, [_VP]),
    "dg_apply_velocity_residual": (ctypes.c_int, [_VP, ctypes.c_int, _VP, _VP, _VP]),
    "dg_batch_workspace_bytes": (ctypes.c_int64, [ctypes.c_int32]),
    "dg_apply_velocity_residual_batched": (ctypes.c_int, [ctypes.POINTER(_VP), ctypes.c_int32, ctypes.c_int,
                                                          ctypes.POINTER(_VP), ctypes.POINTER(_VP), _VP,
                                                          ctypes.c_size_t, _VP]),
    "dg_apply_poisson": (ctypes.c_int, [_VP, ctypes.c_int, _VP, _VP, _VP]),
    "dg_poisson_diagonal": (ctypes.c_int, [_VP, _VP, _VP]),
    "dg_apply_convective": (ctypes.c_int, [_VP, ctypes.c_int, _VP, _VP, _VP]),
    "dg_vorticity_rhs": (ctypes.c_int, [_VP, _VP, _VP, _VP]),
    "dg_vorticity": (ctypes.c_int, [_VP, _VP, _VP, _VP]),
    "dg_pressure_neumann": (ctypes.c_int, [_VP, ctypes.c_int32, ctypes.POINTER(_VP), ctypes.POINTER(_VP),
                                           ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double), _VP,
                                           _VP]),
    "dg_helmholtz_workspace_bytes": (ctypes.c_int64, [_VP, ctypes.POINTER(GmresParams)]),
    "dg_step_workspace_bytes": (ctypes.c_int64, [_VP, ctypes.POINTER(StepParams)]),
    "dg_dual_splitting_step": (ctypes.c_int, [_VP, ctypes.POINTER(StepParams), _VP, _VP, _VP, _VP, _VP,
                                              ctypes.c_size_t, ctypes.POINTER(StepStats), _VP]),
    "dg_solve_helmholtz": (ctypes.c_int, [_VP, _VP, ctypes.c_double, _VP, _VP, ctypes.POINTER(GmresParams), _VP,
                                          ctypes.c_size_t, ctypes.POINTER(GmresStats), _VP]),
    "dg_mg_levels": (ctypes.c_int, [_VP, _VP, ctypes.c_int32]),
    "dg_mg_transfer": (ctypes.c_int, [_VP, ctypes.c_int32, ctypes.c_int32, ctypes.c_int, _VP, _VP, _VP, _VP]),
    "dg_solve_workspace_bytes": (ctypes.c_int64, [_VP, ctypes.POINTER(SolveParams)]),
    "dg_solve_workspace_bytes_for": (ctypes.c_int64, [ctypes.POINTER(MeshParams), ctypes.POINTER(SolveParams)]),
    "dg_solve_poisson": (ctypes.c_int, [_VP, ctypes.POINTER(SolveParams), _VP, _VP, _VP, ctypes.c_size_t,
                                        ctypes.POINTER(SolveStats), _VP]),
    "dg_solve_poisson_noalloc": (ctypes.c_int, [_VP, ctypes.POINTER(SolveParams), _VP, _VP,
                                                ctypes.POINTER(SolveStats), _VP]),
    "dg_solve_batch_workspace_bytes": (ctypes.c_int64, [ctypes.POINTER(_VP), ctypes.c_int32,
                                                       ctypes.POINTER(SolveParams)]),
    "dg_solve_poisson_batched": (ctypes.c_int, [ctypes.POINTER(_VP), ctypes.c_int32, ctypes.POINTER(SolveParams),
                                                ctypes.POINTER(_VP), ctypes.POINTER(_VP), ctypes.POINTER(_VP),
                                                ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(SolveStats),
                                                ctypes.POINTER(ctypes.c_int32), _VP, ctypes.c_size_t, _VP]),
    "dg_last_error": (ctypes.c_char_p, []),
    "dg_build_info": (ctypes.c_char_p, []),
}

_LIB = None


def lib():
    """Load libdgwm.so (raises OSError when it has not been built)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise OSError(f"{LIB_PATH} is missing: build it with paper_1705_08813_amd/build.py "
                          "(or __graft_entry__.build())")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _LIB = L
    return _LIB


def exported_symbols():
    return list(_SIGS)


def check(rc):
    if rc < 0:
        raise DgError(rc, lib().dg_last_error().decode())
    return rc


def params_from(cfg) -> MeshParams:
    d = cfg if isinstance(cfg, dict) else cfg.as_dict()
    p = MeshParams()
    for name, _ in MeshParams._fields_:
        setattr(p, name, d[name])
    return p
