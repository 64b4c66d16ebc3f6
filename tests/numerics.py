"""Error measures shared by the GPU parity tests (no test cases here)."""
import numpy as np

EPS = 2.0 ** -52


def backward_error(A, x, b, babs=None):
    """Normwise backward error of x as a solution of A x = b:
    ||A x - b||_inf / (||A||_inf ||x||_inf + ||b||_inf), with ||babs||_inf in
    place of ||b||_inf when b was formed with cancellation (babs bounds the
    magnitudes of the summands of b).  A backward-stable solve gives a few
    eps times the dimension regardless of the conditioning of A, so this
    catches errors that a conditioning-scaled forward bound lets through."""
    A = np.asarray(A, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.abs(b).max() if babs is None else np.abs(np.asarray(babs)).max()
    den = np.abs(A).sum(1).max() * np.abs(x).max() + nb
    return float(np.abs(A @ x - b).max() / max(den, 1e-300))
