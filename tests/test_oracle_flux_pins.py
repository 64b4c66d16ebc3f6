"""Closed-form pins of the oracle's face terms and of its curved face geometry.

Local Lax-Friedrichs dissipation (Sec. 4.2).  Take a velocity that is constant
in each cell of a fully periodic two-cell box.  Every integral of the residual
then has a closed form:
  - the volume term (grad N_B, -u (x) u) is -u_c (u . n) times the face integral
    of N_B, by the divergence theorem;
  - each face contributes its face integrals of N_B and grad N_B times
    constants.
The component sums are the shortest closed form:
  sum_B r_{0,c,B} = |F| (u0_c - u1_c) (max(2|u0.n|, 2|u1.n|) + 2 tau_F nu).
Both forms are checked.  The 1-D nodal basis, its integrals and its end-point
derivatives come from numpy (Legendre roots and a Vandermonde inverse), not
from the oracle.

Mirror principle on no-slip walls (end of Sec. 4.2).  A constant state has no
jump on interior faces.  At a wall the external state is u+ = -u-, so
  sum_B r_{e,c,B} = |F| 2 u_c (|u.n| + tau_w nu)
with tau_w = wall_ip_mult (k+1)^2 |F| / |Omega_e|.  Flipping the mirror sign
drops the whole right-hand side.

Curved faces (isoparametric cosine lower wall).
  - Closed surface: sum over faces of the integral of n dA is zero.
  - Enclosed volume: sum over faces of the integral of X . n dA is 3 |Omega_e|.
    The face rules integrate both exactly.
  - The lower-wall faces converge to the analytic arc length and normal.
A normal built from J instead of J^{-T}, or a wrong sign, breaks these.
"""
import math

import numpy as np
import pytest
from scipy import integrate

import oracle as O
from paper_1705_08813_amd.inputs import MeshConfig


# ---------------------------------------------------------------- 1-D basis --

def _gl_nodes(n):
    """n Gauss-Lobatto points on [0, 1]: the end points and the roots of P'_{n-1}."""
    inner = np.polynomial.legendre.Legendre.basis(n - 1).deriv().roots() if n > 2 else np.array([])
    t = np.concatenate([[-1.0], np.sort(np.real(inner)), [1.0]])
    return 0.5 * (t + 1.0)


class _Basis1D:
    """Lagrange polynomials through the Gauss-Lobatto points, as monomial
    coefficients (Vandermonde inverse): integrals over [0, 1], values and
    derivatives at the end points."""

    def __init__(self, n):
        x = _gl_nodes(n)
        C = np.linalg.inv(np.vander(x, n, increasing=True))  # L_j(t) = sum_m C[m, j] t^m
        m = np.arange(n)
        self.n = n
        self.integral = (C / (m + 1)[:, None]).sum(0)
        self.val = {0: C[0].copy(), 1: C.sum(0)}
        dC = C[1:] * m[1:, None]
        self.der = {0: dC[0].copy(), 1: dC.sum(0)}


def _face_integrals(bas, h, d, s):
    """Over face (d, s) of a box cell with sizes h: I[B] = int_F N_B dA and
    K[B, k] = int_F d_k N_B dA, nodes B = i + n (j + n m)."""
    n = bas.n
    idx = np.indices((n, n, n)).reshape(3, -1)[::-1]  # idx[a][B] = node index along direction a
    tang = [a for a in range(3) if a != d]
    I = bas.val[s][idx[d]].copy()
    for t in tang:
        I *= h[t] * bas.integral[idx[t]]
    K = np.zeros((n ** 3, 3))
    K[:, d] = bas.der[s][idx[d]] / h[d]
    for t in tang:
        K[:, d] *= h[t] * bas.integral[idx[t]]
    for k in tang:
        (o,) = [t for t in tang if t != k]
        K[:, k] = bas.val[s][idx[d]] * (bas.val[1][idx[k]] - bas.val[0][idx[k]]) * h[o] * bas.integral[idx[o]]
    return I, K


def _cell_sizes(cfg, ey):
    eta = O.vertex_eta(cfg)
    return np.array([cfg.Lx / cfg.nx, eta[ey + 1] - eta[ey], cfg.Lz / cfg.nz])


# ------------------------------------------------------------------- LLF --

@pytest.mark.parametrize("d", [0, 1, 2])
@pytest.mark.parametrize("a,b", [(0.9, -0.3), (0.2, -1.1), (-0.7, -0.25)])
def test_llf_flux_piecewise_constant(d, a, b):
    k = 3
    dims = [1, 1, 1]
    dims[d] = 2
    nu, theta = 0.05, 1.0
    cfg = MeshConfig(nx=dims[0], ny=dims[1], nz=dims[2], k_u=k, nq_u=5, fully_periodic=1, nu=nu, theta=theta)
    n3 = (k + 1) ** 3
    t1, t2 = (d + 1) % 3, (d + 2) % 3
    U = np.zeros((2, 3))
    U[0, d], U[1, d] = a, b
    U[0, t1], U[1, t1] = 0.35, -0.6
    U[0, t2], U[1, t2] = -0.15, 0.45
    u = np.zeros((2, 3, n3))
    for e in range(2):
        for c in range(3):
            u[e, c] = U[e, c]
    r = O.velocity_residual(cfg, u.ravel(), None).reshape(2, 3, n3)

    h = _cell_sizes(cfg, 0)
    area = np.prod(h) / h[d]
    tauF = cfg.ip_factor_u * (k + 1) ** 2 / h[d]
    lam = max(2 * abs(a), 2 * abs(b))
    bas = _Basis1D(k + 1)
    for e in range(2):
        um, up = U[e], U[1 - e]
        jump = um - up
        # component sums: the closed form
        exp_sum = area * jump * (lam + 2 * tauF * nu)
        assert np.abs(r[e].sum(1) - exp_sum).max() < 1e-13 * np.abs(exp_sum).max()
        # node by node: exact face integrals of N_B and grad N_B
        exp = np.zeros((3, n3))
        for s in (0, 1):
            nv = np.zeros(3)
            nv[d] = 1.0 if s else -1.0
            I, K = _face_integrals(bas, h, d, s)
            unm, unp = um @ nv, up @ nv
            for c in range(3):
                fc = 0.5 * (up[c] * unp - um[c] * unm) + (0.5 * lam + tauF * nu) * jump[c]
                Fg = -theta * nu * 0.5 * (jump[c] * nv + jump * nv[c])
                exp[c] += I * fc + K @ Fg
        assert np.abs(r[e] - exp).max() < 1e-13 * np.abs(exp).max()


def test_llf_lambda_is_normal_velocity_only():
    """A tangential velocity of any size leaves Lambda at max(2|u-.n|, 2|u+.n|):
    the jump of the normal component is damped by it alone."""
    k = 2
    nu = 1e-3
    cfg = MeshConfig(nx=2, ny=1, nz=1, k_u=k, nq_u=4, fully_periodic=1, nu=nu)
    n3 = (k + 1) ** 3
    u = np.zeros((2, 3, n3))
    u[0, 0], u[1, 0] = 0.5, 0.1
    u[0, 1], u[1, 1] = 7.0, -9.0   # large tangential velocity
    r = O.velocity_residual(cfg, u.ravel(), None).reshape(2, 3, n3)
    h = _cell_sizes(cfg, 0)
    area = h[1] * h[2]
    tauF = (k + 1) ** 2 / h[0]
    lam = 2 * 0.5
    exp_x = area * (0.5 - 0.1) * (lam + 2 * tauF * nu)
    exp_y = area * (7.0 + 9.0) * (lam + 2 * tauF * nu)
    assert abs(r[0, 0].sum() - exp_x) < 1e-13 * abs(exp_y)
    assert abs(r[0, 1].sum() - exp_y) < 1e-13 * abs(exp_y)


# ------------------------------------------------------------ mirror walls --

@pytest.mark.parametrize("enrich", [0, 1])
@pytest.mark.parametrize("ucon", [(0.6, -0.45, 0.8), (-0.3, 0.9, 0.1)])
def test_mirror_wall_flux_constant_state(enrich, ucon):
    k, nu, theta = 3, 0.05, 1.0
    cfg = MeshConfig(nx=2, ny=3, nz=2, gamma=1.2, k_u=k, nq_u=5, nq_wn=8, enrich_lower=enrich,
                     enrich_upper=enrich, nu=nu, theta=theta)
    n3 = (k + 1) ** 3
    uc = np.asarray(ucon)
    ubar = np.tile(np.repeat(uc, n3), cfg.ncell)
    u = np.concatenate([ubar, np.zeros(3 * cfg.n_enriched)])   # u~ = 0: u = u_bar in every cell
    tau = np.ones(cfg.n_tau)
    r = O.velocity_residual(cfg, u, tau)[: cfg.ncell * 3 * n3].reshape(cfg.ncell, 3, n3)
    ra = O.velocity_residual(cfg, u, tau, absmode=True)
    bas = _Basis1D(k + 1)
    for e in range(cfg.ncell):
        ey = (e // cfg.nx) % cfg.ny
        if ey not in (0, cfg.ny - 1):
            assert np.abs(r[e]).max() < 1e-13 * np.abs(ra).max()   # free stream away from the walls
            continue
        s = 0 if ey == 0 else 1
        h = _cell_sizes(cfg, ey)
        area = h[0] * h[2]
        tau_w = cfg.wall_ip_mult * cfg.ip_factor_u * (k + 1) ** 2 / h[1]
        nv = np.array([0.0, 1.0 if s else -1.0, 0.0])
        un = uc @ nv
        exp_sum = area * 2 * uc * (abs(un) + tau_w * nu)
        assert np.abs(r[e].sum(1) - exp_sum).max() < 1e-13 * np.abs(exp_sum).max()
        I, K = _face_integrals(bas, h, 1, s)
        exp = np.zeros((3, n3))
        for c in range(3):
            fc = 2 * uc[c] * (abs(un) + tau_w * nu)
            Fg = -theta * nu * (uc[c] * nv + uc * nv[c])
            exp[c] = I * fc + K @ Fg
        assert np.abs(r[e] - exp).max() < 1e-13 * np.abs(exp).max()


# ----------------------------------------------------------- curved faces --

CURVED = [
    MeshConfig(nx=4, ny=3, nz=2, wall_amp=0.3, k_u=3, nq_u=5),
    MeshConfig(nx=3, ny=2, nz=1, wall_amp=0.3, k_u=5, nq_u=8),
]


def _volume(cfg, e, nq=8):
    x, w = np.polynomial.legendre.leggauss(nq)
    x, w = 0.5 * (x + 1), 0.5 * w
    vol = 0.0
    for a, wa in zip(x, w):
        for b, wb in zip(x, w):
            _, det = O.cell_map(cfg, e, [a, b, 0.5])   # det J does not depend on z
            vol += abs(det) * wa * wb
    return vol


@pytest.mark.parametrize("cfg", CURVED)
def test_curved_faces_close_and_enclose_the_volume(cfg):
    for e in range(cfg.ncell):
        S = np.zeros(3)
        flux = area = 0.0
        for f in range(6):
            X, nw, w = O.face_points(cfg, e, f)
            S += nw.sum(0)
            flux += (X * nw).sum()
            area += w.sum()
        vol = _volume(cfg, e)
        assert np.abs(S).max() < 2e-14 * area, (e, S)
        assert abs(flux - 3 * vol) < 1e-13 * vol, (e, flux, 3 * vol)


def test_curved_wall_area_and_normal_converge():
    amp, k = 0.3, 3
    Lx, Lz = 2 * math.pi, math.pi

    def dyw(x):
        return -amp * 2 * math.pi / Lx * math.sin(2 * math.pi * x / Lx)

    exact_area = Lz * integrate.quad(lambda x: math.sqrt(1 + dyw(x) ** 2), 0, Lx, epsabs=0, epsrel=1e-13, limit=200)[0]
    area_err, normal_err = [], []
    for nx in (4, 8, 16):
        cfg = MeshConfig(nx=nx, ny=2, nz=1, wall_amp=amp, k_u=k, nq_u=5)
        tot, nerr = 0.0, 0.0
        for ex in range(nx):
            X, nw, w = O.face_points(cfg, ex, 2)   # face (d = 1, s = 0): the lower wall
            tot += w.sum()
            n = nw / w[:, None]
            for x, nn in zip(X[:, 0], n):
                ex_n = np.array([dyw(x), -1.0, 0.0]) / math.sqrt(1 + dyw(x) ** 2)
                nerr = max(nerr, np.abs(nn - ex_n).max())
            assert np.abs(np.linalg.norm(n, axis=1) - 1).max() < 1e-15
        area_err.append(abs(tot - exact_area))
        normal_err.append(nerr)
    assert area_err[0] < 1e-3 * exact_area
    assert area_err[1] < area_err[0] / 2 ** (k + 0.5) and area_err[2] < area_err[1] / 2 ** (k + 0.5)
    assert normal_err[0] < 0.02
    assert normal_err[1] < normal_err[0] / 2 ** (k - 0.5) and normal_err[2] < normal_err[1] / 2 ** (k - 0.5)
