"""Pins for oracle.eig: the Jacobi solver against LAPACK (through NumPy /
SciPy, used here only as an outside reference) and the FD factors against
the textbook p = 1 spectrum."""

import numpy as np
import pytest
import scipy.linalg

from oracle import bspline, eig


@pytest.mark.parametrize("m", [1, 2, 3, 7, 30, 51])
def test_jacobi_matches_lapack(m):
    rng = np.random.default_rng(m)
    A = rng.standard_normal((m, m))
    A = A + A.T
    w, V = eig.jacobi_eigh(A)
    wr = np.linalg.eigvalsh(A)
    np.testing.assert_allclose(w, wr, atol=1e-13 * max(1.0, np.abs(wr).max()))
    np.testing.assert_allclose(V.T @ V, np.eye(m), atol=1e-13)
    np.testing.assert_allclose(A @ V, V * w, atol=1e-12 * max(1.0, np.abs(wr).max()))


def test_jacobi_degenerate_spectrum():
    rng = np.random.default_rng(3)
    Qr, _ = np.linalg.qr(rng.standard_normal((9, 9)))
    lam = np.array([1, 1, 1, 2, 2, 5, 5, 5, 5], float)
    A = Qr @ np.diag(lam) @ Qr.T
    w, V = eig.jacobi_eigh(A)
    np.testing.assert_allclose(w, lam, atol=1e-13)
    np.testing.assert_allclose(A @ V, V * w, atol=1e-13)


def test_cholesky_and_triangular_solves():
    rng = np.random.default_rng(5)
    X = rng.standard_normal((12, 12))
    A = X @ X.T + 12 * np.eye(12)
    L = eig.cholesky(A)
    np.testing.assert_allclose(L, np.linalg.cholesky(A), atol=1e-12)
    B = rng.standard_normal((12, 3))
    np.testing.assert_allclose(eig.solve_lower(L, B), scipy.linalg.solve_triangular(L, B, lower=True), atol=1e-12)
    np.testing.assert_allclose(eig.solve_upper_t(L, B), scipy.linalg.solve_triangular(L.T, B, lower=False), atol=1e-12)
    with pytest.raises(ValueError):
        eig.cholesky(np.diag([1.0, -1.0]))


@pytest.mark.parametrize("p", [1, 2, 3, 5, 8])
def test_pencil_matches_lapack(p):
    K, M = bspline.assemble_dirichlet(9, p)
    lam, Q = eig.gen_eigh(K, M)
    ref = scipy.linalg.eigh(K, M, eigvals_only=True)
    np.testing.assert_allclose(lam, ref, rtol=1e-11)
    np.testing.assert_allclose(Q.T @ M @ Q, np.eye(len(lam)), atol=1e-12)
    np.testing.assert_allclose(Q.T @ K @ Q, np.diag(lam), atol=1e-10 * lam.max())


@pytest.mark.parametrize("n", [5, 16, 33])
def test_fd_p1_closed_form(n):
    """Linear elements: lambda_j = 6(1 - cos t_j) / (h^2 (2 + cos t_j)),
    t_j = j pi / n (the classical finite-element Laplacian spectrum)."""
    K, M = bspline.assemble_dirichlet(n, 1)
    lam, _ = eig.gen_eigh(K, M)
    t = np.arange(1, n) * np.pi / n
    ref = 6 * (1 - np.cos(t)) * n * n / (2 + np.cos(t))
    np.testing.assert_allclose(lam, np.sort(ref), rtol=1e-12)
