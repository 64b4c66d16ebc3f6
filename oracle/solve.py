"""Reference solutions of the singular SIP Poisson system (test infrastructure).

The system A x = b with A symmetric positive semi-definite and null space the
constants (periodic x, z and Neumann walls) has the unique zero-mean solution
x* = A^+ (b - mean(b)).  Two plain references:
  dense_solution: least squares on the dense matrix (tiny meshes),
  cg_solution:    Jacobi-preconditioned conjugate gradients in FP64 calling
                  the C oracle's operator (small meshes), zero-mean projected.
"""
from __future__ import annotations

import numpy as np

from . import dense, poisson_apply, poisson_diag


def project(v):
    return v - v.mean()


def dense_solution(cfg, b):
    A = dense.poisson_matrix(cfg)
    bp = project(np.asarray(b, dtype=float))
    x, *_ = np.linalg.lstsq(A, bp, rcond=1e-13)
    return project(x)


def cg_solution(cfg, b, rtol=1e-13, maxit=20000):
    bp = project(np.asarray(b, dtype=float))
    dinv = 1.0 / poisson_diag(cfg)
    x = np.zeros_like(bp)
    r = bp.copy()
    z = dinv * r
    p = z.copy()
    rz = r @ z
    nb = np.linalg.norm(bp)
    for _ in range(maxit):
        q = poisson_apply(cfg, p)
        a = rz / (p @ q)
        x += a * p
        r -= a * q
        if np.linalg.norm(r) <= rtol * nb:
            break
        z = dinv * r
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
    return project(x)
