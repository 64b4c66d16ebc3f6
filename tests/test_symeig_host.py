"""Host eigendecomposition used for the projection step's per-layer tables
(cyclic Jacobi, csrc/symeig.h), compiled here with g++ into a small driver
and checked against numpy on symmetric matrices with the structure of the
whitened div-div forms (positive semidefinite with a large null space) and on
a general symmetric matrix: A = Z diag(lambda) Z^T, Z^T Z = I, eigenvalues."""
import ctypes
import os
import shutil
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
HDR = os.path.join(HERE, "..", "paper_1705_08813_amd", "csrc", "symeig.h")

DRIVER = r'''
#include "symeig.h"
extern "C" int eig(int n, const double* a, double* lam, double* vt) {
  std::vector<double> A(a, a + (size_t)n * n), L, V;
  const int s = dgwm::sym_eig_jacobi(n, A, L, V);
  for (int i = 0; i < n; ++i) lam[i] = L[i];
  for (size_t i = 0; i < (size_t)n * n; ++i) vt[i] = V[i];
  return s;
}
'''


@pytest.fixture(scope="module")
def eig(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    d = tmp_path_factory.mktemp("symeig")
    src = d / "drv.cpp"
    src.write_text(DRIVER)
    so = d / "drv.so"
    subprocess.run(["g++", "-O2", "-shared", "-fPIC", "-I", os.path.dirname(HDR), str(src), "-o", str(so)],
                   check=True)
    lib = ctypes.CDLL(str(so))
    lib.eig.restype = ctypes.c_int
    lib.eig.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]

    def run(a):
        n = a.shape[0]
        a = np.ascontiguousarray(a, dtype=np.float64)
        lam, vt = np.zeros(n), np.zeros((n, n))
        sweeps = lib.eig(n, a.ctypes.data, lam.ctypes.data, vt.ctypes.data)
        return sweeps, lam, vt.T
    return run


@pytest.mark.parametrize("n,rank", [(81, 60), (192, 150), (6, 6)])
def test_jacobi_matches_numpy(eig, n, rank):
    rng = np.random.default_rng(n)
    F = rng.standard_normal((rank, n)) * np.exp(rng.uniform(-2, 2, n))  # columns of very different scales
    A = F.T @ F
    sweeps, lam, Z = eig(A)
    assert sweeps > 0
    scale = np.abs(A).max()
    assert np.abs(Z @ np.diag(lam) @ Z.T - A).max() <= 1e-12 * scale
    assert np.abs(Z.T @ Z - np.eye(n)).max() <= 1e-12
    ref = np.linalg.eigvalsh(A)
    assert np.abs(np.sort(lam) - ref).max() <= 1e-12 * np.abs(ref).max()
    # the null space (n - rank eigenvalues) comes out at rounding level
    if rank < n:
        assert np.sort(np.abs(lam))[: n - rank].max() <= 1e-12 * np.abs(ref).max()


def test_jacobi_diagonal_and_indefinite(eig):
    d = np.array([3.0, -1.0, 2.0, 0.0])
    sweeps, lam, Z = eig(np.diag(d))
    assert sweeps == 0 and np.array_equal(lam, d) and np.array_equal(Z, np.eye(4))
    rng = np.random.default_rng(3)
    B = rng.standard_normal((40, 40))
    A = B + B.T
    _, lam, Z = eig(A)
    assert np.abs(Z @ np.diag(lam) @ Z.T - A).max() <= 1e-12 * np.abs(A).max()
    assert np.abs(np.sort(lam) - np.linalg.eigvalsh(A)).max() <= 1e-12 * np.abs(A).max()
