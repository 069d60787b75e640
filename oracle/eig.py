"""Dense symmetric eigensolvers without LAPACK.

Test infrastructure only (see the package docstring).

The generalized eigendecompositions of Section 3 (eq:eigendecomposition,
eq:eigedecomposition) and Section 4 (eq:eigendecomposition_reg/out) ask for
an M-orthonormal eigenbasis of a symmetric pencil (K, M) with M SPD.  The
oracle reduces the pencil with a Cholesky factor M = L L^T to the standard
problem C = L^{-1} K L^{-T} and diagonalizes C with the cyclic Jacobi method
(Golub & Van Loan, Matrix Computations, symmetric Schur 2x2 rotation), using
the round-robin ("tournament") ordering so that each round applies m/2
disjoint rotations at once.  Disjoint rotations commute, so a round is
exactly the product of its rotations in any order.
"""

from __future__ import annotations

import numpy as np


def cholesky(A: np.ndarray) -> np.ndarray:
    """Lower-triangular L with A = L L^T (column-by-column, A SPD).
    Raises ValueError if a pivot is not positive."""
    A = np.asarray(A, dtype=np.float64)
    m = A.shape[0]
    L = np.zeros_like(A)
    for j in range(m):
        s = A[j, j] - L[j, :j] @ L[j, :j]
        if not s > 0:
            raise ValueError("matrix is not positive definite")
        L[j, j] = np.sqrt(s)
        L[j + 1:, j] = (A[j + 1:, j] - L[j + 1:, :j] @ L[j, :j]) / L[j, j]
    return L


def solve_lower(L: np.ndarray, B: np.ndarray) -> np.ndarray:
    """Forward substitution L X = B."""
    B = np.asarray(B, dtype=np.float64)
    X = np.zeros_like(B)
    for i in range(L.shape[0]):
        X[i] = (B[i] - L[i, :i] @ X[:i]) / L[i, i]
    return X


def solve_upper_t(L: np.ndarray, B: np.ndarray) -> np.ndarray:
    """Back substitution L^T X = B."""
    B = np.asarray(B, dtype=np.float64)
    m = L.shape[0]
    X = np.zeros_like(B)
    for i in range(m - 1, -1, -1):
        X[i] = (B[i] - L[i + 1:, i] @ X[i + 1:]) / L[i, i]
    return X


def _tournament(m_even: int):
    """Round-robin schedule: m_even-1 rounds, each a perfect matching."""
    players = list(range(m_even))
    rounds = []
    for _ in range(m_even - 1):
        half = m_even // 2
        pairs = [(players[k], players[m_even - 1 - k]) for k in range(half)]
        rounds.append(pairs)
        players = [players[0]] + [players[-1]] + players[1:-1]
    return rounds


def jacobi_eigh(A: np.ndarray, max_sweeps: int = 60):
    """Eigenvalues (ascending) and orthonormal eigenvectors of a symmetric A
    by cyclic Jacobi.  A rotation is skipped when |a_pq| <= eps *
    sqrt(|a_pp a_qq|) (the entry is already negligible at working
    precision); the iteration stops after a sweep that rotates nothing."""
    A = np.array(A, dtype=np.float64, copy=True)
    A = 0.5 * (A + A.T)
    m = A.shape[0]
    V = np.eye(m)
    if m == 1:
        return A.diagonal().copy(), V
    m_even = m + (m % 2)
    rounds = []
    for pairs in _tournament(m_even):
        P = np.array([min(a, b) for a, b in pairs if a < m and b < m], dtype=int)
        Q = np.array([max(a, b) for a, b in pairs if a < m and b < m], dtype=int)
        rounds.append((P, Q))
    eps = np.finfo(np.float64).eps
    tiny = np.finfo(np.float64).tiny
    for _ in range(max_sweeps):
        rotated = False
        for P, Q in rounds:
            app, aqq, apq = A[P, P], A[Q, Q], A[P, Q]
            act = np.abs(apq) > np.maximum(eps * np.sqrt(np.abs(app * aqq)), tiny)
            if not act.any():
                continue
            rotated = True
            P_, Q_ = P[act], Q[act]
            app, aqq, apq = app[act], aqq[act], apq[act]
            theta = (aqq - app) / (2.0 * apq)
            t = np.where(theta >= 0, 1.0, -1.0) / (np.abs(theta) + np.sqrt(theta * theta + 1.0))
            c = 1.0 / np.sqrt(t * t + 1.0)
            s = t * c
            # rows: A <- J^T A
            Ap, Aq = A[P_, :].copy(), A[Q_, :].copy()
            A[P_, :] = c[:, None] * Ap - s[:, None] * Aq
            A[Q_, :] = s[:, None] * Ap + c[:, None] * Aq
            # columns: A <- A J, V <- V J
            Ap, Aq = A[:, P_].copy(), A[:, Q_].copy()
            A[:, P_] = Ap * c - Aq * s
            A[:, Q_] = Ap * s + Aq * c
            Vp, Vq = V[:, P_].copy(), V[:, Q_].copy()
            V[:, P_] = Vp * c - Vq * s
            V[:, Q_] = Vp * s + Vq * c
        if not rotated:
            break
    else:
        raise RuntimeError("Jacobi did not converge")
    w = A.diagonal().copy()
    order = np.argsort(w, kind="stable")
    return w[order], V[:, order]


def gen_eigh(K: np.ndarray, M: np.ndarray):
    """M-orthonormal eigenbasis of the pencil (K, M): returns (lam, Q) with
    K Q = M Q diag(lam), Q^T M Q = I (Section 3, eq:eigendecomposition)."""
    L = cholesky(M)
    C = solve_lower(L, solve_lower(L, K).T).T      # L^{-1} K L^{-T}
    C = 0.5 * (C + C.T)
    lam, Z = jacobi_eigh(C)
    Q = solve_upper_t(L, Z)                         # L^{-T} Z
    return lam, Q
