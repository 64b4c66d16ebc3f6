"""Plain FP64 CPU oracle for the enriched DG velocity residual and the SIP
Poisson operator (arXiv 1705.08813, Sec. 3-4).

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
CPU-baseline leg of the benchmark import this package; the product library
never does, and it shares no code with the HIP path.

The C part (dg_oracle.c) evaluates the operators element by element at every
quadrature point from directly evaluated 1-D Lagrange products.  The Python
modules next to it hold independent cross-checks used as pins:
  dense.py  face-by-face dense assembly of the linear parts on tiny meshes;
  kron.py   Kronecker-sum evaluation of the Poisson operator on box meshes;
  solve.py  reference conjugate-gradient solve.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import build as _build

_LIB = None


class OrcParams(ctypes.Structure):
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
        ("enrich_degree", ctypes.c_int32),
    ]


_D = ctypes.POINTER(ctypes.c_double)
_I64 = ctypes.POINTER(ctypes.c_int64)


def lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(_build.LIB) or os.path.getmtime(_build.LIB) < os.path.getmtime(_build.SRC):
            _build.build()
        L = ctypes.CDLL(_build.LIB)
        P = ctypes.POINTER(OrcParams)
        L.orc_gauss.argtypes = [ctypes.c_int, _D, _D]
        L.orc_gauss_lobatto.argtypes = [ctypes.c_int, _D]
        L.orc_lagrange.argtypes = [ctypes.c_int, _D, ctypes.c_double, _D, _D]
        L.orc_lagrange.restype = None
        L.orc_spalding.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double, _D, _D]
        L.orc_vandriest.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double, _D, _D]
        L.orc_vertex_eta.argtypes = [P, _D]
        L.orc_vertex_eta.restype = None
        L.orc_num_dofs.argtypes = [P, ctypes.c_int]
        L.orc_num_dofs.restype = ctypes.c_int64
        L.orc_num_enriched.argtypes = [P]
        L.orc_num_enriched.restype = ctypes.c_int64
        L.orc_velocity_residual.argtypes = [P, _D, _D, _I64, ctypes.c_int64, _D, ctypes.c_int]
        L.orc_convective_residual.argtypes = [P, _D, _D, _I64, ctypes.c_int64, _D, ctypes.c_int]
        L.orc_poisson_apply.argtypes = [P, _D, _I64, ctypes.c_int64, _D, ctypes.c_int]
        L.orc_poisson_diag.argtypes = [P, _I64, ctypes.c_int64, _D]
        L.orc_psi_point.argtypes = [P, _D, ctypes.c_int64, _D, _D]
        L.orc_velocity_residual_nodal.argtypes = [P, _D, _D, _I64, ctypes.c_int64, _D, ctypes.c_int]
        L.orc_psi_point_nodal.argtypes = [P, _D, ctypes.c_int64, _D, _D]
        L.orc_wall_shear_nodes.argtypes = [P, _D, _D, _D, _D]
        L.orc_psi_volume.argtypes = [P, _D, _D, _I64, ctypes.c_int64, _D]
        L.orc_psi_volume4.argtypes = [P, _D, _D, _I64, ctypes.c_int64, _D]
        L.orc_pressure_gradient.argtypes = [P, _D, _D, _D, _I64, ctypes.c_int64, _D]
        L.orc_divdiv_tau.argtypes = [P, _D, _D, _D, ctypes.c_double, _I64, ctypes.c_int64, _D]
        L.orc_divdiv_apply.argtypes = [P, _D, _D, _D, _D, _I64, ctypes.c_int64, _D]
        L.orc_velocity_divergence.argtypes = [P, _D, _D, _D, _I64, ctypes.c_int64, _D]
        L.orc_enrichment_active.argtypes = [P, _D, _D, ctypes.POINTER(ctypes.c_int32)]
        L.orc_cell_map.argtypes = [P, ctypes.c_int64, _D, _D, _D]
        L.orc_cell_jacobians.argtypes = [P, ctypes.c_int64, ctypes.c_int64, _D, _D]
        L.orc_face_points.argtypes = [P, ctypes.c_int64, ctypes.c_int, _D]
        L.orc_viscous_multiscale.argtypes = [P, _D, _D, _D, _D, ctypes.c_double, ctypes.c_double, ctypes.c_int, _I64,
                                             ctypes.c_int64, _D]
        L.orc_eddy_viscosity_point.argtypes = [P, _D, _D, _D, ctypes.c_double, ctypes.c_double, ctypes.c_int64, _D,
                                               _D]
        L.orc_num_threads.argtypes = []
        L.orc_num_threads.restype = ctypes.c_int
        _LIB = L
    return _LIB


def num_threads() -> int:
    """OpenMP threads the oracle runs on."""
    return int(lib().orc_num_threads())


def params(cfg) -> OrcParams:
    """Oracle parameter struct from a MeshConfig (or any object/dict with the fields)."""
    d = cfg if isinstance(cfg, dict) else cfg.as_dict()
    p = OrcParams()
    for name, _ in OrcParams._fields_:
        setattr(p, name, d.get(name, 0) if name == "enrich_degree" else d[name])
    return p


def require_l0(cfg):
    """The operators other than the velocity residual (and its convective
    form) are built for constant enrichment weights, l = 0 of Sec. 3.1 eq.
    enrichment."""
    d = cfg if isinstance(cfg, dict) else cfg.as_dict()
    if d.get("enrich_degree", 0) != 0:
        raise NotImplementedError("this oracle operator is built for l = 0 enrichment weights only")


def _ptr(a):
    return a.ctypes.data_as(_D)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def gauss(n):
    x = np.zeros(n)
    w = np.zeros(n)
    if lib().orc_gauss(n, _ptr(x), _ptr(w)):
        raise ValueError("bad n")
    return x, w


def gauss_lobatto(n):
    x = np.zeros(n)
    if lib().orc_gauss_lobatto(n, _ptr(x)):
        raise ValueError("bad n")
    return x


def lagrange(nodes, t):
    nodes = _f64(nodes)
    n = len(nodes)
    v = np.zeros(n)
    d = np.zeros(n)
    lib().orc_lagrange(n, _ptr(nodes), float(t), _ptr(v), _ptr(d))
    return v, d


def spalding(yplus, kappa=0.41, B=5.17):
    U = ctypes.c_double()
    dU = ctypes.c_double()
    if lib().orc_spalding(float(yplus), kappa, B, ctypes.byref(U), ctypes.byref(dU)):
        raise ValueError("bad y+")
    return U.value, dU.value


def vandriest(yplus, kappa=0.41, A_plus=26.0):
    """van Driest's law U(y+) (Sec. 3.2, eq. psi) and dU/dy+ by composite Gauss."""
    U = ctypes.c_double()
    dU = ctypes.c_double()
    if lib().orc_vandriest(float(yplus), kappa, A_plus, ctypes.byref(U), ctypes.byref(dU)):
        raise ValueError("bad y+")
    return U.value, dU.value


def vertex_eta(cfg):
    p = params(cfg)
    out = np.zeros(p.ny + 1)
    lib().orc_vertex_eta(ctypes.byref(p), _ptr(out))
    return out


def num_dofs(cfg, field):
    return int(lib().orc_num_dofs(ctypes.byref(params(cfg)), field))


def num_enriched(cfg):
    return int(lib().orc_num_enriched(ctypes.byref(params(cfg))))


def _cells(cfg, cells):
    p = params(cfg)
    if cells is None:
        cells = np.arange(p.nx * p.ny * p.nz, dtype=np.int64)
    return np.ascontiguousarray(cells, dtype=np.int64)


def velocity_residual(cfg, u, tau, cells=None, absmode=False):
    """Residual r for the listed cells (others left zero).  Layout
    [cell][component][node] then [enriched cell][component][enrichment node]
    ((l+1)^3 enrichment nodes: 1 for l = 0, 8 trilinear vertex functions
    for l = 1, node bx + 2 (by + 2 bz))."""
    p = params(cfg)
    u = _f64(u)
    n = num_dofs(cfg, 0)
    if u.size != n:
        raise ValueError(f"u has {u.size} entries, expected {n}")
    tau = _f64(tau) if tau is not None else np.zeros(1)
    cells = _cells(cfg, cells)
    r = np.zeros(n)
    rc = lib().orc_velocity_residual(ctypes.byref(p), _ptr(u), _ptr(tau), cells.ctypes.data_as(_I64),
                                     cells.size, _ptr(r), int(absmode))
    if rc:
        raise RuntimeError(f"orc_velocity_residual failed: {rc}")
    return r


def convective_residual(cfg, u, tau, cells=None, absmode=False):
    """Convective form F^c_e (Sec. 4.2, eq. convstepspat): the velocity
    residual's convective volume and face terms alone (viscous terms, which
    all carry nu, dropped; psi keeps the physical nu).  Layout as
    velocity_residual."""
    p = params(cfg)
    u = _f64(u)
    n = num_dofs(cfg, 0)
    if u.size != n:
        raise ValueError(f"u has {u.size} entries, expected {n}")
    tau = _f64(tau) if tau is not None else np.zeros(1)
    cells = _cells(cfg, cells)
    r = np.zeros(n)
    rc = lib().orc_convective_residual(ctypes.byref(p), _ptr(u), _ptr(tau), cells.ctypes.data_as(_I64),
                                       cells.size, _ptr(r), int(absmode))
    if rc:
        raise RuntimeError(f"orc_convective_residual failed: {rc}")
    return r


def _tau_nodes(cfg, tau_nodes):
    p = params(cfg)
    t = _f64(tau_nodes).reshape(-1)
    if t.size != 2 * p.nz * p.nx:
        raise ValueError(f"tau_nodes has {t.size} entries, expected {2 * p.nz * p.nx}")
    return t


def velocity_residual_nodal(cfg, u, tau_nodes, cells=None, absmode=False):
    """Residual with the nodal wall shear stress field tau_nodes [wall][nz][nx]
    (Sec. 3.2: bilinear tau_w,h, grad psi with the grad tau_w term)."""
    p = params(cfg)
    u = _f64(u)
    n = num_dofs(cfg, 0)
    if u.size != n:
        raise ValueError(f"u has {u.size} entries, expected {n}")
    t = _tau_nodes(cfg, tau_nodes)
    cells = _cells(cfg, cells)
    r = np.zeros(n)
    rc = lib().orc_velocity_residual_nodal(ctypes.byref(p), _ptr(u), _ptr(t), cells.ctypes.data_as(_I64),
                                           cells.size, _ptr(r), int(absmode))
    if rc:
        raise RuntimeError(f"orc_velocity_residual_nodal failed: {rc}")
    return r


def psi_point_nodal(cfg, tau_nodes, e, xi):
    p = params(cfg)
    t = _tau_nodes(cfg, tau_nodes)
    xi = _f64(xi)
    out = np.zeros(4)
    rc = lib().orc_psi_point_nodal(ctypes.byref(p), _ptr(t), int(e), _ptr(xi), _ptr(out))
    if rc:
        raise RuntimeError(f"orc_psi_point_nodal failed: {rc}")
    return out


def wall_shear_nodes(cfg, u, tau=None, tau_nodes=None):
    """Nodal wall shear stress [wall][nz][nx] of the velocity u (Sec. 3.2),
    with psi from the per-point tau or, when given, the nodal tau_nodes."""
    p = params(cfg)
    u = _f64(u)
    if u.size != num_dofs(cfg, 0):
        raise ValueError("u has the wrong size")
    t = _f64(tau) if tau is not None else None
    tn = _tau_nodes(cfg, tau_nodes) if tau_nodes is not None else None
    out = np.zeros(2 * p.nz * p.nx)
    rc = lib().orc_wall_shear_nodes(ctypes.byref(p), _ptr(u), _ptr(t) if t is not None else None,
                                    _ptr(tn) if tn is not None else None, _ptr(out))
    if rc:
        raise RuntimeError(f"orc_wall_shear_nodes failed: {rc}")
    return out.reshape(2, p.nz, p.nx)


def enriched_cells(cfg):
    """Cell indices of the enriched cells, in enrichment order."""
    p = params(cfg)
    out = []
    # enrichment index k = ex + nx (slot + nslots ez): walk k in order
    slots = [] if p.fully_periodic else [ey for ey in range(p.ny) if (ey == 0 and p.enrich_lower)
                                          or (ey == p.ny - 1 and p.enrich_upper)]
    for ez in range(p.nz):
        for ey in slots:
            for ex in range(p.nx):
                out.append(ex + p.nx * (ey + p.ny * ez))
    return np.array(out, dtype=np.int64)


def psi_volume(cfg, cells, tau=None, tau_nodes=None):
    """psi at the enriched volume rule points (x fastest, then the wall-normal
    rule, then z) of the listed enriched cells: [len(cells)][nq_u nq_wn nq_u]."""
    p = params(cfg)
    cells = np.ascontiguousarray(cells, dtype=np.int64)
    t = _f64(tau) if tau is not None else None
    tn = _tau_nodes(cfg, tau_nodes) if tau_nodes is not None else None
    out = np.zeros((cells.size, p.nq_u * p.nq_wn * p.nq_u))
    rc = lib().orc_psi_volume(ctypes.byref(p), _ptr(t) if t is not None else None,
                              _ptr(tn) if tn is not None else None, cells.ctypes.data_as(_I64), cells.size,
                              _ptr(out))
    if rc:
        raise RuntimeError(f"orc_psi_volume failed: {rc}")
    return out


def pressure_gradient(cfg, p, tau=None, tau_nodes=None, cells=None):
    """Pressure gradient term (Sec. 4.2) g(v) = -(div v, p)_e + (v . n, {{p}})
    for every velocity test function (velocity layout); psi from the per-point
    tau or the nodal tau_nodes."""
    pr = params(cfg)
    p = _f64(p)
    if p.size != num_dofs(cfg, 1):
        raise ValueError("p has the wrong size")
    t = _f64(tau) if tau is not None else None
    tn = _tau_nodes(cfg, tau_nodes) if tau_nodes is not None else None
    cells = _cells(cfg, cells)
    out = np.zeros(num_dofs(cfg, 0))
    rc = lib().orc_pressure_gradient(ctypes.byref(pr), _ptr(p), _ptr(t) if t is not None else None,
                                     _ptr(tn) if tn is not None else None, cells.ctypes.data_as(_I64), cells.size,
                                     _ptr(out))
    if rc:
        raise RuntimeError(f"orc_pressure_gradient failed: {rc}")
    return out


def velocity_divergence(cfg, u, tau=None, tau_nodes=None, cells=None):
    """Velocity divergence term (Sec. 4.2) c(q) = -(grad q, u)_e + (q, {{u}} . n)
    for every pressure test function (pressure layout)."""
    pr = params(cfg)
    u = _f64(u)
    if u.size != num_dofs(cfg, 0):
        raise ValueError("u has the wrong size")
    t = _f64(tau) if tau is not None else None
    tn = _tau_nodes(cfg, tau_nodes) if tau_nodes is not None else None
    cells = _cells(cfg, cells)
    out = np.zeros(num_dofs(cfg, 1))
    rc = lib().orc_velocity_divergence(ctypes.byref(pr), _ptr(u), _ptr(t) if t is not None else None,
                                       _ptr(tn) if tn is not None else None, cells.ctypes.data_as(_I64), cells.size,
                                       _ptr(out))
    if rc:
        raise RuntimeError(f"orc_velocity_divergence failed: {rc}")
    return out


def divdiv_tau(cfg, u, dt_over_cr, tau=None, tau_nodes=None, cells=None):
    """tau_D per cell (Sec. 4.2, eq. tauD): volume-averaged |u| times the cube
    root of the cell volume times dt/Cr."""
    pr = params(cfg)
    u = _f64(u)
    if u.size != num_dofs(cfg, 0):
        raise ValueError("u has the wrong size")
    t = _f64(tau) if tau is not None else None
    tn = _tau_nodes(cfg, tau_nodes) if tau_nodes is not None else None
    cells = _cells(cfg, cells)
    out = np.zeros(pr.nx * pr.ny * pr.nz)
    rc = lib().orc_divdiv_tau(ctypes.byref(pr), _ptr(u), _ptr(t) if t is not None else None,
                              _ptr(tn) if tn is not None else None, float(dt_over_cr), cells.ctypes.data_as(_I64),
                              cells.size, _ptr(out))
    if rc:
        raise RuntimeError(f"orc_divdiv_tau failed: {rc}")
    return out


def divdiv_apply(cfg, u, tau_d, tau=None, tau_nodes=None, cells=None):
    """Div-div penalty (Sec. 4.2, eq. div-div) D(v, u) = (div v, tau_D div u)_e for
    every velocity test function (velocity layout)."""
    pr = params(cfg)
    u = _f64(u)
    td = _f64(tau_d)
    if u.size != num_dofs(cfg, 0) or td.size != pr.nx * pr.ny * pr.nz:
        raise ValueError("u or tau_d has the wrong size")
    t = _f64(tau) if tau is not None else None
    tn = _tau_nodes(cfg, tau_nodes) if tau_nodes is not None else None
    cells = _cells(cfg, cells)
    out = np.zeros(num_dofs(cfg, 0))
    rc = lib().orc_divdiv_apply(ctypes.byref(pr), _ptr(u), _ptr(t) if t is not None else None,
                                _ptr(tn) if tn is not None else None, _ptr(td), cells.ctypes.data_as(_I64),
                                cells.size, _ptr(out))
    if rc:
        raise RuntimeError(f"orc_divdiv_apply failed: {rc}")
    return out


def psi_volume4(cfg, cells, tau=None, tau_nodes=None):
    """psi and grad psi at the enriched volume rule points of the listed
    enriched cells: [len(cells)][points][4]."""
    p = params(cfg)
    cells = np.ascontiguousarray(cells, dtype=np.int64)
    t = _f64(tau) if tau is not None else None
    tn = _tau_nodes(cfg, tau_nodes) if tau_nodes is not None else None
    out = np.zeros((cells.size, p.nq_u * p.nq_wn * p.nq_u, 4))
    rc = lib().orc_psi_volume4(ctypes.byref(p), _ptr(t) if t is not None else None,
                               _ptr(tn) if tn is not None else None, cells.ctypes.data_as(_I64), cells.size,
                               _ptr(out))
    if rc:
        raise RuntimeError(f"orc_psi_volume4 failed: {rc}")
    return out


def enrichment_active(cfg, tau=None, tau_nodes=None):
    """Switch-off rule (Sec. 3.2): 1 where the enrichment of an enriched cell
    is on, in enrichment order."""
    p = params(cfg)
    t = _f64(tau) if tau is not None else None
    tn = _tau_nodes(cfg, tau_nodes) if tau_nodes is not None else None
    out = np.zeros(num_enriched(cfg), dtype=np.int32)
    rc = lib().orc_enrichment_active(ctypes.byref(p), _ptr(t) if t is not None else None,
                                     _ptr(tn) if tn is not None else None,
                                     out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    if rc:
        raise RuntimeError(f"orc_enrichment_active failed: {rc}")
    return out


def poisson_apply(cfg, x, cells=None, absmode=False):
    p = params(cfg)
    x = _f64(x)
    n = num_dofs(cfg, 1)
    if x.size != n:
        raise ValueError(f"x has {x.size} entries, expected {n}")
    cells = _cells(cfg, cells)
    y = np.zeros(n)
    rc = lib().orc_poisson_apply(ctypes.byref(p), _ptr(x), cells.ctypes.data_as(_I64), cells.size, _ptr(y),
                                 int(absmode))
    if rc:
        raise RuntimeError(f"orc_poisson_apply failed: {rc}")
    return y


def poisson_diag(cfg, cells=None):
    p = params(cfg)
    cells = _cells(cfg, cells)
    d = np.zeros(num_dofs(cfg, 1))
    rc = lib().orc_poisson_diag(ctypes.byref(p), cells.ctypes.data_as(_I64), cells.size, _ptr(d))
    if rc:
        raise RuntimeError(f"orc_poisson_diag failed: {rc}")
    return d


def psi_point(cfg, tau, e, xi):
    p = params(cfg)
    tau = _f64(tau)
    xi = _f64(xi)
    out = np.zeros(4)
    rc = lib().orc_psi_point(ctypes.byref(p), _ptr(tau), int(e), _ptr(xi), _ptr(out))
    if rc:
        raise RuntimeError(f"orc_psi_point failed: {rc}")
    return out


def cell_map(cfg, e, xi):
    p = params(cfg)
    xi = _f64(xi)
    X = np.zeros(3)
    det = ctypes.c_double()
    lib().orc_cell_map(ctypes.byref(p), int(e), _ptr(xi), _ptr(X), ctypes.byref(det))
    return X, det.value


def cell_jacobians(cfg, e, pts):
    """J[q][d][a] = dX_d / dxi_a of cell e at the reference points pts (npts, 3)."""
    p = params(cfg)
    pts = np.ascontiguousarray(pts, dtype=np.float64)
    J = np.zeros((len(pts), 3, 3))
    rc = lib().orc_cell_jacobians(ctypes.byref(p), int(e), len(pts), _ptr(pts), _ptr(J))
    if rc:
        raise RuntimeError(f"orc_cell_jacobians failed: {rc}")
    return J


def face_points(cfg, e, f):
    """Quadrature points of face f = 2 d + s of cell e (the velocity residual's
    face rule): X [npts, 3], n w dA [npts, 3] and w dA [npts]."""
    p = params(cfg)
    out = np.zeros(7 * 16 * 16)
    n = lib().orc_face_points(ctypes.byref(p), int(e), int(f), _ptr(out))
    if n < 0:
        raise ValueError(f"orc_face_points failed: {n}")
    o = out[: 7 * n].reshape(n, 7)
    return o[:, :3].copy(), o[:, 3:6].copy(), o[:, 6].copy()


C_DES, BETA = 0.85, 6.0   # Sec. 2.2, eq. ydes: calibrated C_DES and the smoothing exponent


def viscous_multiscale(cfg, u, u_nut=None, tau=None, tau_nodes=None, c_des=C_DES, beta=BETA, clip=True, cells=None):
    """A u = -F^nu_e of Sec. 4.2, eq. viscous_multiscale, for every velocity test
    function (velocity layout); nu_t from the enrichment coefficients of u_nut
    (default: u).  clip=False drops the limit of eq. minvt (pins only)."""
    p = params(cfg)
    u = _f64(u)
    n = num_dofs(cfg, 0)
    if u.size != n:
        raise ValueError("u has the wrong size")
    un = u if u_nut is None else _f64(u_nut)
    if un.size != n:
        raise ValueError("u_nut has the wrong size")
    t = _f64(tau) if tau is not None else None
    tn = _tau_nodes(cfg, tau_nodes) if tau_nodes is not None else None
    cells = _cells(cfg, cells)
    r = np.zeros(n)
    rc = lib().orc_viscous_multiscale(ctypes.byref(p), _ptr(u), _ptr(un), _ptr(t) if t is not None else None,
                                      _ptr(tn) if tn is not None else None, float(c_des), float(beta), int(clip),
                                      cells.ctypes.data_as(_I64), cells.size, _ptr(r))
    if rc:
        raise RuntimeError(f"orc_viscous_multiscale failed: {rc}")
    return r


def eddy_viscosity_point(cfg, u_nut, e, xi, tau=None, tau_nodes=None, c_des=C_DES, beta=BETA):
    """(nu_t, y, y+, |eps(u~)|) at reference point xi of enriched cell e (Sec. 2.2, eqs. mix, lmix, ydes)."""
    p = params(cfg)
    un = _f64(u_nut)
    t = _f64(tau) if tau is not None else None
    tn = _tau_nodes(cfg, tau_nodes) if tau_nodes is not None else None
    out = np.zeros(4)
    rc = lib().orc_eddy_viscosity_point(ctypes.byref(p), _ptr(un), _ptr(t) if t is not None else None,
                                        _ptr(tn) if tn is not None else None, float(c_des), float(beta), int(e),
                                        _ptr(_f64(xi)), _ptr(out))
    if rc:
        raise RuntimeError(f"orc_eddy_viscosity_point failed: {rc}")
    return out
