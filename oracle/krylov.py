"""Preconditioned conjugate gradients and the CG-Lanczos condition estimate.

Test infrastructure only (see the package docstring).

Section 3 solves A u = f by PCG; Section 7 fixes the protocol: zero initial
guess, stop when the relative residual reaches 1e-8.  Readings where the
paper is silent: the residual norm is the unpreconditioned Euclidean norm of
the recursively updated residual, ||r_k||_2 <= tol ||f||_2, and the reported
iteration count is the number of solution updates made until the test first
passes (so an exact preconditioner gives 1 iteration).

The Lanczos matrix is rebuilt from the PCG coefficients with the classical
CG-Lanczos relation (Saad, Iterative Methods for Sparse Linear Systems,
Section 6.7.3): T_jj = 1/alpha_j + beta_{j-1}/alpha_{j-1},
T_{j,j+1} = sqrt(beta_j)/alpha_j.  Its extreme eigenvalues estimate those of
P^{-1} A, whose ratio is the condition number of Proposition 1.
"""

from __future__ import annotations

import numpy as np

from . import eig


def pcg(apply_A, apply_Pinv, f: np.ndarray, tol: float = 1e-8, maxit: int = 500):
    """Returns (u, iterations, converged, relres_history, alphas, betas)."""
    f = np.asarray(f, dtype=np.float64)
    u = np.zeros_like(f)
    r = f.copy()
    nf = np.sqrt(np.vdot(f, f))
    hist = [1.0]
    alphas, betas = [], []
    if nf == 0.0:
        return u, 0, True, hist, alphas, betas
    z = apply_Pinv(r)
    p = z.copy()
    rz = np.vdot(r, z)
    for it in range(1, maxit + 1):
        q = apply_A(p)
        pq = np.vdot(p, q)
        alpha = rz / pq
        u = u + alpha * p
        r = r - alpha * q
        alphas.append(alpha)
        rel = np.sqrt(np.vdot(r, r)) / nf
        hist.append(rel)
        if rel <= tol:
            return u, it, True, hist, alphas, betas
        z = apply_Pinv(r)
        rz_new = np.vdot(r, z)
        beta = rz_new / rz
        betas.append(beta)
        p = z + beta * p
        rz = rz_new
    return u, maxit, False, hist, alphas, betas


def lanczos_tridiag(alphas, betas) -> np.ndarray:
    """Symmetric tridiagonal T_k from k PCG steps (needs len(betas) >= k-1)."""
    k = len(alphas)
    T = np.zeros((k, k))
    for j in range(k):
        T[j, j] = 1.0 / alphas[j]
        if j > 0:
            T[j, j] += betas[j - 1] / alphas[j - 1]
        if j + 1 < k:
            T[j, j + 1] = T[j + 1, j] = np.sqrt(betas[j]) / alphas[j]
    return T


def kappa_estimate(alphas, betas):
    """(lambda_min, lambda_max, kappa) of the Lanczos matrix."""
    k = min(len(alphas), len(betas) + 1)
    T = lanczos_tridiag(alphas[:k], betas[:k - 1])
    w, _ = eig.jacobi_eigh(T)
    return w[0], w[-1], w[-1] / w[0]
