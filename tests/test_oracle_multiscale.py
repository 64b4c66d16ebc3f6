"""Pins of the oracle's multiscale viscous operator (Sec. 4.2, eq.
viscous_multiscale) and of its eddy viscosity (Sec. 2.2, eqs. mix, lmix, ydes).

- Energy identity.  With v = u, the adjoint and consistency face terms of
  every face class cancel (the skew-symmetric construction behind the
  coercivity argument of Sec. 4.3).  So u^T A u equals the volume energy
      sum_e (eps(u_bar), 2 nu eps(u_bar)) + (eps(u_bar), 2 nuhat eps(u~))
            + (eps(u~), 2 (nu + nu_t) eps(u~))
  plus the penalty energy  sum_F tau nu |[u]|^2  (2 tau nu |u|^2 on walls).
  Both are computed here in numpy: Vandermonde basis, face traces
  assembled face by face, psi and nu_t at the points from the separately
  pinned point functions.  A wrong row mask, weight or sign in any face term
  breaks the identity.
- Reduction.  With u~ = 0 and nu_t = 0 the polynomial rows are the SIP
  viscous operator with adjoint sign theta = -1.  Those are the v_bar,u_bar
  row of the equation, which the dense-assembly pins cover.
- Coercivity (Sec. 4.3, eq. minvt).  With the limit nuhat =
  min(nu + nu_t, 2 sqrt(nu (nu + nu_t))) the symmetric part of A is positive
  semi-definite for any nu_t field, here at nu_t/nu up to about 60.
- The eddy viscosity at a point against its closed form.  With l = 0,
  grad u~ = ut (x) grad psi, so |eps(u~)| = sqrt(|ut|^2 |grad psi|^2 + (ut . grad psi)^2).
- Degree-1 enrichment weights (Sec. 3.1 eq. enrichment, l = 1): the energy
  identity with u~ = psi sum_B N_B ut_B evaluated here from the trilinear
  vertex functions, the reduction to l = 0 when the eight coefficients of
  every component are equal (the vertex functions sum to one), and the eddy
  viscosity from grad u~ = sum_B ut_B (x) (N_B grad psi + psi grad N_B).
"""
import math

import numpy as np
import pytest

import oracle as O
from paper_1705_08813_amd.inputs import MeshConfig, Workload, draw_inputs


def _gl_nodes(n):
    inner = np.polynomial.legendre.Legendre.basis(n - 1).deriv().roots() if n > 2 else np.array([])
    t = np.concatenate([[-1.0], np.sort(np.real(inner)), [1.0]])
    return 0.5 * (t + 1.0)


class _Basis:
    """Tensor Lagrange basis through the Gauss-Lobatto points (Vandermonde)."""

    def __init__(self, n):
        self.n = n
        self.C = np.linalg.inv(np.vander(_gl_nodes(n), n, increasing=True))

    def line(self, t):
        m = np.arange(self.n)
        v = (t ** m) @ self.C
        dm = np.concatenate([[0.0], m[1:] * t ** (m[1:] - 1)])
        return v, dm @ self.C

    def at(self, xi, h):
        """N_B and grad N_B (physical, box cell of sizes h), B = i + n (j + n m)."""
        (vx, dx), (vy, dy), (vz, dz) = (self.line(xi[a]) for a in range(3))
        val = np.einsum("m,j,i->mji", vz, vy, vx).ravel()
        g = np.stack([np.einsum("m,j,i->mji", vz, vy, dx).ravel() / h[0],
                      np.einsum("m,j,i->mji", vz, dy, vx).ravel() / h[1],
                      np.einsum("m,j,i->mji", dz, vy, vx).ravel() / h[2]], axis=1)
        return val, g


def _vertex(xi, h):
    """Trilinear vertex functions N_B (B = bx + 2 (by + 2 bz)) and their
    physical gradients on a box cell of sizes h."""
    N = np.zeros(8)
    dN = np.zeros((8, 3))
    for B in range(8):
        bits = (B & 1, (B >> 1) & 1, B >> 2)
        f = [xi[d] if bits[d] else 1.0 - xi[d] for d in range(3)]
        df = [(1.0 if bits[d] else -1.0) / h[d] for d in range(3)]
        N[B] = f[0] * f[1] * f[2]
        dN[B] = [df[0] * f[1] * f[2], f[0] * df[1] * f[2], f[0] * f[1] * df[2]]
    return N, dN


def _enr_grad(coef, ps, xi, h):
    """u~ and grad u~ [c][d] from coefficients coef (3, nle) and psi, grad psi."""
    if coef.shape[1] == 1:
        return ps[0] * coef[:, 0], np.outer(coef[:, 0], ps[1:])
    N, dN = _vertex(xi, h)
    return ps[0] * coef @ N, coef @ (N[:, None] * ps[None, 1:] + ps[0] * dN)


def _gauss(n):
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (x + 1), 0.5 * w


class _Field:
    """u = u_bar + psi ut at reference points of the cells of a flat channel."""

    def __init__(self, cfg, u, u_nut, tau):
        self.cfg, self.u, self.u_nut, self.tau = cfg, u, u_nut, tau
        self.n3 = (cfg.k_u + 1) ** 3
        self.bas = _Basis(cfg.k_u + 1)
        self.eta = O.vertex_eta(cfg)
        self.enr = {int(e): k for k, e in enumerate(O.enriched_cells(cfg))}

    def h(self, e):
        ey = (e // self.cfg.nx) % self.cfg.ny
        return np.array([self.cfg.Lx / self.cfg.nx, self.eta[ey + 1] - self.eta[ey], self.cfg.Lz / self.cfg.nz])

    def eval(self, e, xi):
        """u_bar, grad u_bar, u~, grad u~, nu_t at xi of cell e."""
        val, g = self.bas.at(xi, self.h(e))
        ub = np.array([val @ self.u[(e * 3 + c) * self.n3:(e * 3 + c + 1) * self.n3] for c in range(3)])
        gb = np.array([g.T @ self.u[(e * 3 + c) * self.n3:(e * 3 + c + 1) * self.n3] for c in range(3)])
        ut, gt, nut = np.zeros(3), np.zeros((3, 3)), 0.0
        k = self.enr.get(e)
        if k is not None:
            nle = (getattr(self.cfg, "enrich_degree", 0) + 1) ** 3
            off = self.cfg.ncell * 3 * self.n3 + 3 * nle * k
            coef = self.u[off:off + 3 * nle].reshape(3, nle)
            ps = O.psi_point(self.cfg, self.tau, e, xi)
            ut, gt = _enr_grad(coef, ps, xi, self.h(e))
            nut = O.eddy_viscosity_point(self.cfg, self.u_nut, e, xi, tau=self.tau)[0]
        return ub, gb, ut, gt, nut


def _sym(g):
    return 0.5 * (g + g.T)


def _energies(cfg, u, u_nut, tau):
    """Volume and penalty energies of u, assembled in numpy."""
    F = _Field(cfg, u, u_nut, tau)
    nu = cfg.nu
    n = cfg.k_u + 1
    qu, wu = _gauss(cfg.nq_u)
    qw, ww = _gauss(cfg.nq_wn)
    e_vol = 0.0
    for e in range(cfg.ncell):
        h = F.h(e)
        ry = (qw, ww) if e in F.enr else (qu, wu)
        for z, wz in zip(qu, wu):
            for y, wy in zip(*ry):
                for x, wx in zip(qu, wu):
                    ub, gb, ut, gt, nut = F.eval(e, (x, y, z))
                    eb, et = _sym(gb), _sym(gt)
                    nt = nu + nut
                    nhat = min(nt, 2 * math.sqrt(nu * nt))
                    dens = np.sum(eb * 2 * nu * eb) + np.sum(eb * 2 * nhat * et) + np.sum(et * 2 * nt * et)
                    e_vol += wx * wy * wz * np.prod(h) * dens
    e_pen = 0.0
    nx, ny, nz = cfg.nx, cfg.ny, cfg.nz
    for e in range(cfg.ncell):
        ex, ey, ez = e % nx, (e // nx) % ny, e // (nx * ny)
        h = F.h(e)
        for d in range(3):
            idx = [ex, ey, ez]
            dims = [nx, ny, nz]
            j = idx[d] + 1
            wall = d == 1 and j >= ny
            if d == 1 and ey == 0:
                # the lower wall face of this cell
                faces = [(0, None)]
            else:
                faces = []
            if wall:
                faces.append((1, None))
            else:
                idx[d] = j % dims[d]
                faces.append((1, idx[0] + nx * (idx[1] + ny * idx[2])))
            t1, t2 = [a for a in range(3) if a != d]
            for s, nb in faces:
                # tangential rules: the larger of the two cells' rules
                def rule(a):
                    big = a == 1 and (e in F.enr or (nb is not None and nb in F.enr))
                    return (qw, ww) if big else (qu, wu)
                (q1, w1), (q2, w2) = rule(t1), rule(t2)
                tauF = cfg.ip_factor_u * n ** 2 / h[d]
                if nb is not None:
                    tauF = cfg.ip_factor_u * n ** 2 * max(1 / h[d], 1 / F.h(nb)[d])
                else:
                    tauF *= cfg.wall_ip_mult
                area = h[t1] * h[t2]
                for a, wa in zip(q1, w1):
                    for b, wb in zip(q2, w2):
                        xi = np.zeros(3)
                        xi[d], xi[t1], xi[t2] = s, a, b
                        ub, _, ut, _, _ = F.eval(e, xi)
                        um = ub + ut
                        if nb is None:
                            jmp2 = 4 * um @ um / 2  # tau nu u-.(2 u-) from the wall's only side
                        else:
                            xn = xi.copy()
                            xn[d] = 0.0
                            ubp, _, utp, _, _ = F.eval(nb, xn)
                            jmp = um - (ubp + utp)
                            jmp2 = jmp @ jmp
                        e_pen += wa * wb * area * tauF * nu * jmp2
    return e_vol, e_pen


MS_CASES = {
    # both walls enriched, stretched; wall-cell tops at y+ ~ 60-120, nu_t / nu up to ~15
    "k2_both": (MeshConfig(nx=2, ny=3, nz=2, gamma=1.0, k_u=2, nq_u=4, nq_wn=8, nu=1.0 / 400), 31),
    # one enriched wall, k = 3, a wall-normal rule of 6 points
    "k3_lower": (MeshConfig(nx=2, ny=3, nz=2, gamma=0.6, k_u=3, nq_u=5, nq_wn=6, nu=1.0 / 300, enrich_upper=0), 32),
    # degree-1 enrichment weights, both walls
    "k2_both_l1": (MeshConfig(nx=2, ny=3, nz=2, gamma=1.0, k_u=2, nq_u=4, nq_wn=8, nu=1.0 / 400, enrich_degree=1), 39),
}


@pytest.mark.parametrize("name", list(MS_CASES))
def test_energy_identity_skew_face_terms_cancel(name):
    cfg, seed = MS_CASES[name]
    inp = draw_inputs(Workload("ms", cfg, seed, 0.5, 1.5))
    u = inp["u"]
    u_nut = np.random.default_rng(seed + 100).uniform(-1, 1, cfg.n_vel)
    r = O.viscous_multiscale(cfg, u, u_nut=u_nut, tau=inp["tau"])
    e_vol, e_pen = _energies(cfg, u, u_nut, inp["tau"])
    got = u @ r
    assert e_vol > 0 and e_pen > 0
    assert abs(got - (e_vol + e_pen)) <= 1e-12 * (e_vol + e_pen), (got, e_vol, e_pen)


def test_reduction_to_sip_without_rans_scale():
    cfg = MeshConfig(nx=2, ny=3, nz=2, gamma=1.0, k_u=3, nq_u=5, nq_wn=8, nu=1.0 / 400, theta=-1.0)
    inp = draw_inputs(Workload("ms", cfg, 33, 0.5, 1.5))
    n = cfg.ncell * 3 * (cfg.k_u + 1) ** 3
    u = inp["u"].copy()
    u[n:] = 0.0   # u~ = 0
    r = O.viscous_multiscale(cfg, u, u_nut=u, tau=inp["tau"])  # and nu_t = 0
    V = 2 * O.velocity_residual(cfg, u, inp["tau"]) - 0.5 * O.velocity_residual(cfg, 2 * u, inp["tau"])
    assert np.abs(r[:n] - V[:n]).max() <= 1e-12 * np.abs(V[:n]).max()
    # without enrichment every row is the SIP operator
    plain = cfg.with_(enrich_lower=0, enrich_upper=0)
    up = inp["u"][:n]
    r = O.viscous_multiscale(plain, up)
    V = 2 * O.velocity_residual(plain, up, None) - 0.5 * O.velocity_residual(plain, 2 * up, None)
    assert np.abs(r - V).max() <= 1e-12 * np.abs(V).max()


def test_linear_in_u_for_fixed_eddy_viscosity():
    cfg, seed = MS_CASES["k2_both"]
    inp = draw_inputs(Workload("ms", cfg, seed, 0.5, 1.5))
    rng = np.random.default_rng(34)
    a, b, un = rng.uniform(-1, 1, (3, cfg.n_vel))
    ra = O.viscous_multiscale(cfg, a, u_nut=un, tau=inp["tau"])
    rb = O.viscous_multiscale(cfg, b, u_nut=un, tau=inp["tau"])
    rab = O.viscous_multiscale(cfg, 2 * a - 3 * b, u_nut=un, tau=inp["tau"])
    assert np.abs(rab - (2 * ra - 3 * rb)).max() <= 1e-12 * np.abs(rab).max()


def _dense(cfg, u_nut, tau, clip):
    n = cfg.n_vel
    A = np.zeros((n, n))
    for j in range(n):
        x = np.zeros(n)
        x[j] = 1.0
        A[:, j] = O.viscous_multiscale(cfg, x, u_nut=u_nut, tau=tau, clip=clip)
    return A


def test_coercivity_with_the_eddy_viscosity_limit():
    cfg = MeshConfig(nx=2, ny=2, nz=1, gamma=0.8, k_u=2, nq_u=4, nq_wn=8, nu=1.0 / 400)
    inp = draw_inputs(Workload("ms", cfg, 35, 0.5, 1.5))
    u_nut = np.zeros(cfg.n_vel)
    u_nut[cfg.ncell * 3 * 27:] = np.random.default_rng(36).uniform(2, 4, 3 * cfg.n_enriched)  # large nu_t
    cells = O.enriched_cells(cfg)
    nuts = [O.eddy_viscosity_point(cfg, u_nut, e, (0.5, 0.7, 0.5), tau=inp["tau"])[0] for e in cells]
    assert max(nuts) / cfg.nu > 20
    A = _dense(cfg, u_nut, inp["tau"], clip=True)
    ev = np.linalg.eigvalsh(0.5 * (A + A.T))
    assert ev[0] >= -1e-12 * ev[-1], (ev[0], ev[-1])


def test_eddy_viscosity_closed_form():
    cfg, seed = MS_CASES["k2_both"]
    inp = draw_inputs(Workload("ms", cfg, seed, 0.5, 1.5))
    u_nut = np.random.default_rng(37).uniform(-1, 1, cfg.n_vel)
    eta = O.vertex_eta(cfg)
    n3 = (cfg.k_u + 1) ** 3
    enr = O.enriched_cells(cfg)
    for k, e in enumerate(enr[[0, len(enr) - 1]]):
        kk = 0 if k == 0 else len(enr) - 1
        ey = (e // cfg.nx) % cfg.ny
        hy = eta[ey + 1] - eta[ey]
        ut = u_nut[cfg.ncell * 3 * n3 + 3 * kk: cfg.ncell * 3 * n3 + 3 * kk + 3]
        for xi in ((0.2, 0.1, 0.7), (0.9, 0.6, 0.3), (0.5, 1.0, 0.5), (0.4, 0.0, 0.8)):
            got = O.eddy_viscosity_point(cfg, u_nut, e, xi, tau=inp["tau"])
            ps = O.psi_point(cfg, inp["tau"], e, xi)
            y_phys = eta[ey] + hy * xi[1]
            y = 1 - abs(y_phys)
            xq, _ = _gauss(cfg.nq_u)
            qx, qz = int(np.argmin(abs(xq - xi[0]))), int(np.argmin(abs(xq - xi[2])))
            w = 0 if ey == 0 else 1
            tw = inp["tau"].reshape(2, cfg.nz, cfg.nx, cfg.nq_u, cfg.nq_u)[w, e // (cfg.nx * cfg.ny), e % cfg.nx, qz, qx]
            yp = y * math.sqrt(tw) / cfg.nu
            ch = O.C_DES * hy / (cfg.k_u + 1)
            ydes = 0.0 if y == 0 else (y ** -O.BETA + ch ** -O.BETA) ** (-1 / O.BETA)
            lmix = cfg.kappa * ydes * (1 - math.exp(-yp / cfg.A_plus))
            g = ps[1:]
            eps = math.sqrt((ut @ ut) * (g @ g) + (ut @ g) ** 2)
            assert abs(got[1] - y) <= 1e-15 and abs(got[2] - yp) <= 1e-12 * max(yp, 1)
            assert abs(got[3] - eps) <= 1e-13 * eps
            assert abs(got[0] - lmix ** 2 * eps) <= 1e-13 * max(lmix ** 2 * eps, 1e-300)


def test_harmonic_weights_on_inner_enriched_faces():
    """Two enriched wall cells side by side (periodic in x, so they share both x
    faces), u_bar = 0, u~ only in cell 0, different eddy viscosities.  Seen from
    cell 1 every face term vanishes except, on the shared faces,
      -{{(nu + nu_t) (grad u~ + grad u~^T)}}_w n - tau nu psi+ ut+
    and the harmonic weights (eq. harmweights) make the first term
    nu_H (grad u~+ + grad u~+^T) n with
    nu_H = (nu + nu_t-)(nu + nu_t+) / (2 nu + nu_t- + nu_t+).
    The component sums of cell 1's polynomial rows are the face integrals of
    that (sum_B N_B = 1)."""
    cfg = MeshConfig(nx=2, ny=3, nz=1, gamma=1.0, k_u=2, nq_u=4, nq_wn=8, nu=1.0 / 400, enrich_upper=0)
    inp = draw_inputs(Workload("ms", cfg, 38, 0.5, 1.5))
    n3 = 27
    off = cfg.ncell * 3 * n3
    u = np.zeros(cfg.n_vel)
    u[off:off + 3] = [0.7, -0.4, 0.3]            # u~ in cell 0 only
    u_nut = np.zeros(cfg.n_vel)
    u_nut[off:off + 3] = [2.0, 1.0, -0.5]       # nu_t in cell 0
    u_nut[off + 3:off + 6] = [0.2, -0.1, 0.05]  # a smaller nu_t in cell 1
    r = O.viscous_multiscale(cfg, u, u_nut=u_nut, tau=inp["tau"])
    F = _Field(cfg, u, u_nut, inp["tau"])
    nu = cfg.nu
    h = F.h(1)
    tauF = cfg.ip_factor_u * 9 / h[0]
    qy, wy = _gauss(cfg.nq_wn)
    qz, wz = _gauss(cfg.nq_u)
    exp = np.zeros(3)
    for s in (0, 1):              # cell 1's faces x = 0 and x = 1, both shared with cell 0
        nv = np.array([1.0 if s else -1.0, 0.0, 0.0])
        for y, wyy in zip(qy, wy):
            for z, wzz in zip(qz, wz):
                _, _, _, _, num = F.eval(1, (float(s), y, z))
                _, _, utp, gtp, nup = F.eval(0, (1.0 - s, y, z))
                nuH = (nu + num) * (nu + nup) / (2 * nu + num + nup)
                Sn = (gtp + gtp.T) @ nv
                exp += wyy * wzz * h[1] * h[2] * (-nuH * Sn - tauF * nu * utp)   # [u] = 0 - u~+
    got = r[3 * n3:6 * n3].reshape(3, n3).sum(1)
    assert np.abs(got - exp).max() <= 1e-12 * np.abs(exp).max(), (got, exp)
    # the weights matter here: with equal weights the result would differ
    assert abs(u_nut[off] - u_nut[off + 3]) > 1


@pytest.mark.parametrize("name", ["k2_both", "k3_lower"])
def test_l1_equal_weights_reduce_to_l0(name):
    cfg0, seed = MS_CASES[name]
    cfg1 = cfg0.with_(enrich_degree=1)
    inp = draw_inputs(Workload("ms", cfg0, seed, 0.5, 1.5))
    n = cfg0.ncell * 3 * (cfg0.k_u + 1) ** 3
    un0 = np.random.default_rng(seed + 200).uniform(-1, 1, cfg0.n_vel)

    def rep8(v):
        return np.concatenate([v[:n], np.repeat(v[n:].reshape(-1, 3)[:, :, None], 8, axis=2).ravel()])

    r0 = O.viscous_multiscale(cfg0, inp["u"], u_nut=un0, tau=inp["tau"])
    r1 = O.viscous_multiscale(cfg1, rep8(inp["u"]), u_nut=rep8(un0), tau=inp["tau"])
    scale = np.abs(r0).max()
    assert np.abs(r1[:n] - r0[:n]).max() <= 1e-13 * scale
    assert np.abs(r1[n:].reshape(-1, 3, 8).sum(axis=2) - r0[n:].reshape(-1, 3)).max() <= 1e-13 * scale


def test_l1_eddy_viscosity_closed_form():
    cfg, seed = MS_CASES["k2_both_l1"]
    inp = draw_inputs(Workload("ms", cfg, seed, 0.5, 1.5))
    u_nut = np.random.default_rng(40).uniform(-1, 1, cfg.n_vel)
    eta = O.vertex_eta(cfg)
    n3 = (cfg.k_u + 1) ** 3
    enr = O.enriched_cells(cfg)
    for kk in (0, len(enr) - 1):
        e = int(enr[kk])
        ey = (e // cfg.nx) % cfg.ny
        h = np.array([cfg.Lx / cfg.nx, eta[ey + 1] - eta[ey], cfg.Lz / cfg.nz])
        coef = u_nut[cfg.ncell * 3 * n3 + 24 * kk: cfg.ncell * 3 * n3 + 24 * kk + 24].reshape(3, 8)
        for xi in ((0.2, 0.1, 0.7), (0.9, 0.6, 0.3), (0.4, 0.0, 0.8)):
            got = O.eddy_viscosity_point(cfg, u_nut, e, xi, tau=inp["tau"])
            ps = O.psi_point(cfg, inp["tau"], e, xi)
            _, gt = _enr_grad(coef, ps, xi, h)
            eps = math.sqrt(2.0 * np.sum(_sym(gt) ** 2))
            assert abs(got[3] - eps) <= 1e-13 * eps
            ch = O.C_DES * h[1] / (cfg.k_u + 1)
            y = got[1]
            ydes = 0.0 if y == 0 else (y ** -O.BETA + ch ** -O.BETA) ** (-1 / O.BETA)
            lmix = cfg.kappa * ydes * (1 - math.exp(-got[2] / cfg.A_plus))
            assert abs(got[0] - lmix ** 2 * eps) <= 1e-13 * max(lmix ** 2 * eps, 1e-300)
