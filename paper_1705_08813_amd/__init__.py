"""MI355X (gfx950) library for the enriched DG operators of the multiscale
RANS/LES wall model of Krank, Kronbichler & Wall (arXiv 1705.08813).

The compute path is the HIP shared library libdgwm.so (C ABI in
include/dgwm.h).  This package holds its Python binding (argument
marshalling over torch device memory and streams), the seeded input
generators, and the build script.  Importing the package does not load the
library; creating a Mesh does, and fails loudly if it is missing.
"""
from __future__ import annotations

import ctypes

from . import _lib
from ._lib import DG_F32, DG_F64, DgError, SolveParams, SolveStats

__all__ = ["Mesh", "DgError", "DG_F64", "DG_F32", "SolveParams", "SolveStats", "apply_velocity_residual_batched",
           "batch_workspace", "solve_poisson_batched", "solve_batch_workspace"]


def _stream_ptr(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dptr(t):
    return ctypes.c_void_p(t.data_ptr())


class Mesh:
    """One channel instance resident on the current device.

    cfg: a MeshConfig (paper_1705_08813_amd.inputs) or dict with the fields of
    dg_mesh_params.  tau_w: host array of wall shear stresses per wall-face
    Gauss point (layout of include/dgwm.h) or None for tau_w = 1.
    """

    def __init__(self, cfg, tau_w=None, device=None, stream=None):
        import numpy as np
        import torch
        L = _lib.lib()
        self.cfg = cfg
        self.params = _lib.params_from(cfg)
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        nbytes = _lib.check(L.dg_mesh_workspace_bytes(ctypes.byref(self.params)))
        self.workspace = torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=self.device)
        tau_ptr = None
        if tau_w is not None:
            self._tau_host = np.ascontiguousarray(tau_w, dtype=np.float64)
            tau_ptr = self._tau_host.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        handle = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _lib.check(L.dg_setup_mesh(ctypes.byref(self.params), tau_ptr, _dptr(self.workspace), nbytes,
                                       _stream_ptr(stream), ctypes.byref(handle)))
        self.handle = handle
        self.n_vel = int(L.dg_num_dofs(handle, 0))
        self.n_p = int(L.dg_num_dofs(handle, 1))
        self.n_enriched = int(L.dg_num_enriched(handle))

    # ------------------------------------------------------------------
    def _check_vec(self, t, n, name):
        import torch
        if not isinstance(t, torch.Tensor) or t.device != self.device or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous tensor on {self.device}")
        if t.numel() != n:
            raise ValueError(f"{name} has {t.numel()} entries, expected {n}")
        if t.dtype not in (torch.float64, torch.float32):
            raise ValueError(f"{name} must be float64 or float32")
        return DG_F64 if t.dtype == torch.float64 else DG_F32

    def apply_velocity_residual(self, u, r=None, stream=None):
        import torch
        prec = self._check_vec(u, self.n_vel, "u")
        if r is None:
            r = torch.empty_like(u)
        if self._check_vec(r, self.n_vel, "r") != prec:
            raise ValueError("u and r must have the same dtype")
        _lib.check(_lib.lib().dg_apply_velocity_residual(self.handle, prec, _dptr(u), _dptr(r), _stream_ptr(stream)))
        return r

    def apply_convective(self, u, r=None, stream=None):
        """dg_apply_convective: the convective part of the velocity residual."""
        import torch
        prec = self._check_vec(u, self.n_vel, "u")
        if r is None:
            r = torch.empty_like(u)
        if self._check_vec(r, self.n_vel, "r") != prec:
            raise ValueError("u and r must have the same dtype")
        _lib.check(_lib.lib().dg_apply_convective(self.handle, prec, _dptr(u), _dptr(r), _stream_ptr(stream)))
        return r

    def apply_poisson(self, p, y=None, stream=None):
        import torch
        prec = self._check_vec(p, self.n_p, "p")
        if y is None:
            y = torch.empty_like(p)
        if self._check_vec(y, self.n_p, "y") != prec:
            raise ValueError("p and y must have the same dtype")
        _lib.check(_lib.lib().dg_apply_poisson(self.handle, prec, _dptr(p), _dptr(y), _stream_ptr(stream)))
        return y

    def poisson_diagonal(self, stream=None):
        import torch
        d = torch.empty(self.n_p, dtype=torch.float64, device=self.device)
        _lib.check(_lib.lib().dg_poisson_diagonal(self.handle, _dptr(d), _stream_ptr(stream)))
        return d

    def mg_levels(self):
        """dg_mg_levels: [(nx, ny, nz, cx, cy, cz)] of every multigrid level."""
        n = _lib.check(_lib.lib().dg_mg_levels(self.handle, None, 0))
        buf = (ctypes.c_int32 * (6 * max(n, 1)))()
        _lib.check(_lib.lib().dg_mg_levels(self.handle, buf, n))
        return [tuple(buf[6 * l:6 * l + 6]) for l in range(n)]

    def mg_transfer(self, level, direction, x, add=None, out=None, stream=None):
        """dg_mg_transfer: direction 0 restricts x (level `level`) to level
        level+1; direction 1 prolongs x (level level+1) and adds `add`
        (zeros when None) on level `level`.  float64 or float32 tensors."""
        import torch
        lv = self.mg_levels()
        if not 0 <= level < len(lv) - 1:
            raise ValueError("level outside the hierarchy")
        np3 = (self.cfg.k_p + 1) ** 3
        nf = lv[level][0] * lv[level][1] * lv[level][2] * np3
        nc = lv[level + 1][0] * lv[level + 1][1] * lv[level + 1][2] * np3
        n_in, n_out = (nf, nc) if direction == 0 else (nc, nf)
        if x.dtype not in (torch.float64, torch.float32):
            raise ValueError("x must be float64 or float32")
        prec = 0 if x.dtype == torch.float64 else 1
        for t, n, name in ((x, n_in, "x"), (add, n_out, "add"), (out, n_out, "out")):
            if t is not None and (t.dtype != x.dtype or t.device != self.device or not t.is_contiguous()
                                  or t.numel() != n):
                raise ValueError(f"{name} must be a contiguous {x.dtype} tensor of {n} entries on {self.device}")
        if out is None:
            out = torch.empty(n_out, dtype=x.dtype, device=self.device)
        if direction == 1 and add is None:
            add = torch.zeros(n_out, dtype=x.dtype, device=self.device)
        _lib.check(_lib.lib().dg_mg_transfer(self.handle, level, direction, prec, _dptr(x),
                                             _dptr(add) if add is not None else None, _dptr(out),
                                             _stream_ptr(stream)))
        return out

    def _check_f64(self, t, n, name):
        import torch
        if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or t.device != self.device \
                or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous float64 tensor on {self.device}")
        if t.numel() != n:
            raise ValueError(f"{name} has {t.numel()} entries, expected {n}")

    @property
    def n_tau(self):
        p = self.params
        return 2 * p.nz * p.nx * p.nq_u * p.nq_u

    @property
    def n_wall_nodes(self):
        return 2 * self.params.nz * self.params.nx

    def update_wall_shear(self, tau_dev, stream=None):
        """Per-point tau_w (device, [wall][ez][ex][qz][qx]); recomputes psi."""
        self._check_f64(tau_dev, self.n_tau, "tau")
        _lib.check(_lib.lib().dg_update_wall_shear(self.handle, _dptr(tau_dev), _stream_ptr(stream)))

    def wall_shear_nodes(self, u, out=None, stream=None):
        """Nodal wall shear stress of both walls from the FP64 velocity u,
        returned as a (2, nz, nx) float64 device tensor."""
        import torch
        self._check_f64(u, self.n_vel, "u")
        if out is None:
            out = torch.empty((2, self.params.nz, self.params.nx), dtype=torch.float64, device=self.device)
        self._check_f64(out, self.n_wall_nodes, "out")
        _lib.check(_lib.lib().dg_wall_shear_nodes(self.handle, _dptr(u), _dptr(out), _stream_ptr(stream)))
        return out

    def update_wall_shear_nodes(self, tau_nodes, stream=None):
        """Nodal tau_w (device, [wall][jz][jx]); recomputes psi with the
        bilinear wall field."""
        self._check_f64(tau_nodes, self.n_wall_nodes, "tau_nodes")
        _lib.check(_lib.lib().dg_update_wall_shear_nodes(self.handle, _dptr(tau_nodes), _stream_ptr(stream)))

    def project_velocity(self, u_old, u_new=None, stream=None):
        """L2 projection (eq. l2) of u_old from the space before the last
        wall-shear update onto the current one; returns u_new (u_new may be
        u_old: in place)."""
        import torch
        self._check_f64(u_old, self.n_vel, "u_old")
        if u_new is None:
            u_new = torch.empty_like(u_old)
        self._check_f64(u_new, self.n_vel, "u_new")
        _lib.check(_lib.lib().dg_project_velocity(self.handle, _dptr(u_old), _dptr(u_new), _stream_ptr(stream)))
        return u_new

    def apply_inverse_mass(self, r, x=None, stream=None):
        """x = M^{-1} r with the velocity mass matrix (x may be r)."""
        import torch
        self._check_f64(r, self.n_vel, "r")
        if x is None:
            x = torch.empty_like(r)
        self._check_f64(x, self.n_vel, "x")
        _lib.check(_lib.lib().dg_apply_inverse_mass(self.handle, _dptr(r), _dptr(x), _stream_ptr(stream)))
        return x

    def apply_pressure_gradient(self, p, g=None, stream=None):
        """Pressure gradient term P p (velocity layout, Sec. 4.2)."""
        import torch
        self._check_f64(p, self.n_p, "p")
        if g is None:
            g = torch.empty(self.n_vel, dtype=torch.float64, device=self.device)
        self._check_f64(g, self.n_vel, "g")
        _lib.check(_lib.lib().dg_apply_pressure_gradient(self.handle, _dptr(p), _dptr(g), _stream_ptr(stream)))
        return g

    def apply_velocity_divergence(self, u, c=None, stream=None):
        """Velocity divergence term C u (pressure layout, Sec. 4.2)."""
        import torch
        self._check_f64(u, self.n_vel, "u")
        if c is None:
            c = torch.empty(self.n_p, dtype=torch.float64, device=self.device)
        self._check_f64(c, self.n_p, "c")
        _lib.check(_lib.lib().dg_apply_velocity_divergence(self.handle, _dptr(u), _dptr(c), _stream_ptr(stream)))
        return c

    @property
    def n_cells(self):
        p = self.params
        return p.nx * p.ny * p.nz

    def divdiv_tau(self, u, dt_over_cr, tau_d=None, stream=None):
        """Per-cell div-div penalty parameter tau_D (Sec. 4.2, eq. tauD)."""
        import torch
        self._check_f64(u, self.n_vel, "u")
        if tau_d is None:
            tau_d = torch.empty(self.n_cells, dtype=torch.float64, device=self.device)
        self._check_f64(tau_d, self.n_cells, "tau_d")
        _lib.check(_lib.lib().dg_divdiv_tau(self.handle, _dptr(u), float(dt_over_cr), _dptr(tau_d),
                                            _stream_ptr(stream)))
        return tau_d

    def apply_divdiv(self, tau_d, u, out=None, stream=None):
        """Div-div penalty D u (Sec. 4.2, eq. div-div), velocity layout."""
        import torch
        self._check_f64(tau_d, self.n_cells, "tau_d")
        self._check_f64(u, self.n_vel, "u")
        if out is None:
            out = torch.empty_like(u)
        self._check_f64(out, self.n_vel, "out")
        _lib.check(_lib.lib().dg_apply_divdiv(self.handle, _dptr(tau_d), _dptr(u), _dptr(out), _stream_ptr(stream)))
        return out

    def projection_step(self, tau_d, u_hat, g, scale, x=None, stream=None):
        """Element-wise projection step (Sec. 4.2): (M + D) x = M u_hat - scale g."""
        import torch
        self._check_f64(tau_d, self.n_cells, "tau_d")
        self._check_f64(u_hat, self.n_vel, "u_hat")
        self._check_f64(g, self.n_vel, "g")
        if x is None:
            x = torch.empty_like(u_hat)
        self._check_f64(x, self.n_vel, "x")
        _lib.check(_lib.lib().dg_projection_step(self.handle, _dptr(tau_d), _dptr(u_hat), _dptr(g), float(scale),
                                                 _dptr(x), _stream_ptr(stream)))
        return x

    def eddy_viscosity(self, u, c_des=0.85, beta=6.0, nut=None, stream=None):
        """nu_t of the RANS scale at every enriched quadrature point (Sec. 2.2),
        from the enrichment coefficients of u (float64 device tensor)."""
        import torch
        self._check_f64(u, self.n_vel, "u")
        n = _lib.check(_lib.lib().dg_eddy_viscosity_points(self.handle))
        if nut is None:
            nut = torch.empty(max(int(n), 1), dtype=torch.float64, device=self.device)
        _lib.check(_lib.lib().dg_eddy_viscosity(self.handle, _dptr(u), float(c_des), float(beta), _dptr(nut),
                                                _stream_ptr(stream)))
        return nut[:n]

    def apply_viscous_multiscale(self, nut, u, out=None, stream=None):
        """out = A u, the multiscale viscous operator of Sec. 4.2 (FP64)."""
        import torch
        self._check_f64(u, self.n_vel, "u")
        if out is None:
            out = torch.empty_like(u)
        self._check_f64(out, self.n_vel, "out")
        _lib.check(_lib.lib().dg_apply_viscous_multiscale(self.handle, _dptr(nut) if nut is not None else None,
                                                          _dptr(u), _dptr(out), _stream_ptr(stream)))
        return out

    def enrichment_active(self, stream=None):
        """Activity flags (int32 device tensor, 1 on / 0 switched off) of the
        enriched cells in the current space."""
        import torch
        out = torch.empty(max(self.n_enriched, 1), dtype=torch.int32, device=self.device)
        _lib.check(_lib.lib().dg_enrichment_active(self.handle, _dptr(out), _stream_ptr(stream)))
        return out[:self.n_enriched]

    def vorticity_rhs(self, u, b=None, stream=None):
        """dg_vorticity_rhs: b(v) = (v, curl u)_e."""
        import torch
        self._check_f64(u, self.n_vel, "u")
        b = torch.empty_like(u) if b is None else b
        self._check_f64(b, self.n_vel, "b")
        _lib.check(_lib.lib().dg_vorticity_rhs(self.handle, _dptr(u), _dptr(b), _stream_ptr(stream)))
        return b

    def vorticity(self, u, omega=None, stream=None):
        """dg_vorticity: the L2 projection of curl u onto the velocity space."""
        import torch
        self._check_f64(u, self.n_vel, "u")
        omega = torch.empty_like(u) if omega is None else omega
        self._check_f64(omega, self.n_vel, "omega")
        _lib.check(_lib.lib().dg_vorticity(self.handle, _dptr(u), _dptr(omega), _stream_ptr(stream)))
        return omega

    def pressure_neumann(self, us, omegas, betas, f=(0.0, 0.0, 0.0), rhs=None, stream=None):
        """dg_pressure_neumann: adds the wall term of the high-order pressure
        Neumann data into rhs (zeros when None) and returns it."""
        import torch
        nh = len(us)
        if nh != len(omegas) or nh != len(betas) or nh not in (1, 2):
            raise ValueError("one or two (u, omega, beta) time levels")
        for t in list(us) + list(omegas):
            self._check_f64(t, self.n_vel, "u/omega")
        rhs = torch.zeros(self.n_p, dtype=torch.float64, device=self.device) if rhs is None else rhs
        self._check_f64(rhs, self.n_p, "rhs")
        VP = ctypes.c_void_p
        up = (VP * nh)(*[u.data_ptr() for u in us])
        op = (VP * nh)(*[o.data_ptr() for o in omegas])
        bp = (ctypes.c_double * nh)(*[float(b) for b in betas])
        fp = (ctypes.c_double * 3)(*[float(v) for v in f])
        _lib.check(_lib.lib().dg_pressure_neumann(self.handle, nh, up, op, bp, fp, _dptr(rhs), _stream_ptr(stream)))
        return rhs

    def solve_helmholtz(self, nut, gamma0_over_dt, b, x=None, rtol=1e-12, max_iter=500, restart=30, workspace=None,
                        stream=None):
        """dg_solve_helmholtz: (gamma0/dt) M x + A(nut) x = (gamma0/dt) M b by
        restarted GMRES; returns (x, GmresStats)."""
        import torch
        self._check_f64(b, self.n_vel, "b")
        if x is None:
            x = b.clone()
        self._check_f64(x, self.n_vel, "x")
        gp = _lib.GmresParams(rtol=rtol, max_iter=max_iter, restart=restart)
        if workspace is None:
            nb = _lib.check(_lib.lib().dg_helmholtz_workspace_bytes(self.handle, ctypes.byref(gp)))
            workspace = torch.empty(int(nb), dtype=torch.uint8, device=self.device)
        st = _lib.GmresStats()
        _lib.check(_lib.lib().dg_solve_helmholtz(self.handle, _dptr(nut) if nut is not None else None,
                                                 float(gamma0_over_dt), _dptr(b), _dptr(x), ctypes.byref(gp),
                                                 _dptr(workspace), workspace.numel(), ctypes.byref(st),
                                                 _stream_ptr(stream)))
        return x, st

    def step_params(self, dt, order=2, f=(0.0, 0.0, 0.0), dt_over_cr=None, poisson=None, helmholtz_rtol=1e-10,
                    helmholtz_max_iter=1000, helmholtz_restart=30, c_des=0.85, beta_des=6.0):
        """dg_step_params with the constant-step BDF/extrapolation coefficients
        of order 1 or 2 (gamma0 = 3/2, alpha = (2, -1/2), beta = (2, -1) for
        order 2); dt_over_cr defaults to dt / 0.14 (the paper's Courant number)."""
        if order == 2:
            g0, al, be = 1.5, (2.0, -0.5), (2.0, -1.0)
        elif order == 1:
            g0, al, be = 1.0, (1.0, 0.0), (1.0, 0.0)
        else:
            raise ValueError("order must be 1 or 2")
        sp = poisson if poisson is not None else self.solve_params(rtol=1e-10, mixed=True)
        return _lib.StepParams(dt=dt, gamma0=g0, alpha=(ctypes.c_double * 2)(*al), beta=(ctypes.c_double * 2)(*be),
                               order=order, f=(ctypes.c_double * 3)(*f),
                               dt_over_cr=dt / 0.14 if dt_over_cr is None else dt_over_cr, c_des=c_des,
                               beta_des=beta_des, poisson=sp,
                               helmholtz=_lib.GmresParams(rtol=helmholtz_rtol, max_iter=helmholtz_max_iter,
                                                          restart=helmholtz_restart))

    def dual_splitting_step(self, sp, u_n, u_nm1, p, u_np1=None, workspace=None, stream=None):
        """dg_dual_splitting_step: returns (u_np1, p, StepStats); p is updated in place."""
        import torch
        self._check_f64(u_n, self.n_vel, "u_n")
        if sp.order == 2:
            self._check_f64(u_nm1, self.n_vel, "u_nm1")
        self._check_f64(p, self.n_p, "p")
        u_np1 = torch.empty_like(u_n) if u_np1 is None else u_np1
        self._check_f64(u_np1, self.n_vel, "u_np1")
        if workspace is None:
            nb = _lib.check(_lib.lib().dg_step_workspace_bytes(self.handle, ctypes.byref(sp)))
            workspace = torch.empty(int(nb), dtype=torch.uint8, device=self.device)
        st = _lib.StepStats()
        _lib.check(_lib.lib().dg_dual_splitting_step(self.handle, ctypes.byref(sp), _dptr(u_n),
                                                     _dptr(u_nm1) if u_nm1 is not None else None, _dptr(u_np1),
                                                     _dptr(p), _dptr(workspace), workspace.numel(), ctypes.byref(st),
                                                     _stream_ptr(stream)))
        return u_np1, p, st

    def solve_params(self, rtol=1e-10, mixed=True, max_outer=2000, max_inner=0, cheb_degree=5,
                     multigrid=True, coarse_degree=3):
        return SolveParams(rtol=rtol, max_outer=max_outer, max_inner=max_inner, cheb_degree=cheb_degree,
                           mixed=int(mixed), multigrid=int(multigrid),
                           coarse_degree=coarse_degree)

    def solve_workspace(self, sp):
        import torch
        n = _lib.check(_lib.lib().dg_solve_workspace_bytes(self.handle, ctypes.byref(sp)))
        return torch.empty(max(int(n), 256), dtype=torch.uint8, device=self.device)

    def solve_poisson(self, b, x=None, sp=None, workspace=None, stream=None):
        import torch
        if sp is None:
            sp = self.solve_params()
        if b.dtype != torch.float64:
            raise ValueError("b must be float64")
        self._check_vec(b, self.n_p, "b")
        if x is None:
            x = torch.zeros_like(b)
        self._check_vec(x, self.n_p, "x")
        if workspace is None:
            workspace = self.solve_workspace(sp)
        st = SolveStats()
        _lib.check(_lib.lib().dg_solve_poisson(self.handle, ctypes.byref(sp), _dptr(b), _dptr(x), _dptr(workspace),
                                               workspace.numel(), ctypes.byref(st), _stream_ptr(stream)))
        return x, st

    def solve_poisson_noalloc(self, b, x=None, sp=None, stream=None):
        """dg_solve_poisson_noalloc: the solve with the library's built-in
        per-GPU workspace (no workspace argument, nothing allocated)."""
        import torch
        if sp is None:
            sp = self.solve_params()
        if b.dtype != torch.float64:
            raise ValueError("b must be float64")
        self._check_vec(b, self.n_p, "b")
        if x is None:
            x = torch.zeros_like(b)
        self._check_vec(x, self.n_p, "x")
        st = SolveStats()
        _lib.check(_lib.lib().dg_solve_poisson_noalloc(self.handle, ctypes.byref(sp), _dptr(b), _dptr(x),
                                                       ctypes.byref(st), _stream_ptr(stream)))
        return x, st

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            _lib.lib().dg_destroy_mesh(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def batch_workspace(n, device=None):
    """Device workspace for a batched velocity call over n meshes."""
    import torch
    nbytes = _lib.check(_lib.lib().dg_batch_workspace_bytes(int(n)))
    dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=dev)


def solve_batch_workspace(meshes, sp):
    """Device descriptor workspace of a batched solve over these meshes."""
    import torch
    n = len(meshes)
    hs = (ctypes.c_void_p * n)(*[m.handle.value for m in meshes])
    nbytes = _lib.check(_lib.lib().dg_solve_batch_workspace_bytes(hs, n, ctypes.byref(sp)))
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=meshes[0].device)


def solve_poisson_batched(meshes, bs, xs=None, sp=None, workspaces=None, batch_ws=None, stream=None):
    """dg_solve_poisson_batched: the solves of every mesh of the list
    advanced together.  Returns (xs, stats, codes): per mesh solution,
    SolveStats and status code (0 = converged)."""
    import torch
    n = len(meshes)
    if n == 0 or len(bs) != n or (xs is not None and len(xs) != n):
        raise ValueError("meshes, bs and xs must be non-empty lists of one length")
    if sp is None:
        sp = meshes[0].solve_params()
    if xs is None:
        xs = [torch.zeros_like(b) for b in bs]
    for m, b, x in zip(meshes, bs, xs):
        if b.dtype != torch.float64 or x.dtype != torch.float64:
            raise ValueError("b and x must be float64")
        m._check_vec(b, m.n_p, "b")
        m._check_vec(x, m.n_p, "x")
    if workspaces is None:
        workspaces = [m.solve_workspace(sp) for m in meshes]
    if batch_ws is None:
        batch_ws = solve_batch_workspace(meshes, sp)
    VP = ctypes.c_void_p
    hs = (VP * n)(*[m.handle.value for m in meshes])
    bp = (VP * n)(*[b.data_ptr() for b in bs])
    xp = (VP * n)(*[x.data_ptr() for x in xs])
    wp = (VP * n)(*[w.data_ptr() for w in workspaces])
    wb = (ctypes.c_size_t * n)(*[w.numel() for w in workspaces])
    stats = (SolveStats * n)()
    codes = (ctypes.c_int32 * n)()
    _lib.check(_lib.lib().dg_solve_poisson_batched(hs, n, ctypes.byref(sp), bp, xp, wp, wb, stats, codes,
                                                   _dptr(batch_ws), batch_ws.numel(), _stream_ptr(stream)))
    return xs, list(stats), list(codes)


def apply_velocity_residual_batched(meshes, us, rs=None, workspace=None, stream=None):
    """r_i = R_i(u_i) for every mesh of the list in one batched call
    (bit-for-bit the single-mesh result).  All vectors share one dtype."""
    import torch
    n = len(meshes)
    if n == 0 or len(us) != n or (rs is not None and len(rs) != n):
        raise ValueError("meshes, us and rs must be non-empty lists of one length")
    if rs is None:
        rs = [torch.empty_like(u) for u in us]
    prec = None
    for m, u, r in zip(meshes, us, rs):
        pu = m._check_vec(u, m.n_vel, "u")
        if m._check_vec(r, m.n_vel, "r") != pu or (prec is not None and pu != prec):
            raise ValueError("every u and r of a batch must have one dtype")
        prec = pu
    if workspace is None:
        workspace = batch_workspace(n, meshes[0].device)
    VP = ctypes.c_void_p
    hs = (VP * n)(*[m.handle.value for m in meshes])
    up = (VP * n)(*[u.data_ptr() for u in us])
    rp = (VP * n)(*[r.data_ptr() for r in rs])
    _lib.check(_lib.lib().dg_apply_velocity_residual_batched(hs, n, prec, up, rp, _dptr(workspace),
                                                             workspace.numel(), _stream_ptr(stream)))
    return rs

