"""The IFFD preconditioner on [0,1]^d with homogeneous Dirichlet conditions
on every face (D_k = {0,1}), built two independent ways, plus the classical
Fast Diagonalization (FD) it approximates.

Test infrastructure only (see the package docstring).

Notation (per direction; all directions share n and p here)
    m      = n + p - 2            dim S_{p,h,{0,1}}                 (Section 2)
    n_reg  = n-1 (p odd), n (p even);  n_out = p-1 (odd), p-2 (even)
                                                            (eq:reg_space_dim)
    K, M   1-D stiffness and mass on S_{p,h,{0,1}}                 (Section 3)

What the preconditioner is (Proposition 1, eq:preconditioner2)
    P = sum_k  M x .. x Ktilde (slot k) x .. x M,
    Ktilde = Qt^{-T} Lt Qt^{-1}, where Qt = [V_reg Q_reg, V_out Q_out] and
    Lt = blkdiag(L_reg, L_out) come from the restricted pencils
    (eq:eigendecomposition_reg/out).  The proof of Corollary 1 shows
    v^T Ktilde v = v_reg^T K v_reg + v_out^T K v_out for v = v_reg + v_out, so
    Ktilde = Pr^T K Pr + Po^T K Po with Po the M-orthogonal projector onto
    S^out and Pr = I - Po.  Ktilde depends only on the splitting, hence P^{-1}r
    is uniquely defined whatever bases are picked for S^reg and S^out.

Route A (from the definitions)
    S^reg = null(E), E = the even-derivative conditions of eq:reg_space at
    x = 0 and x = 1 (orders 2, 4, .., 2*floor((p-1)/2)); S^out its L2
    complement, spanned by M^{-1} E^T (reading of the V_out formula of
    Section 4: the printed formula lies inside range(V_reg,0) and would not be
    M-orthogonal to S^reg); Ktilde as above; (Lt, Qt) = Jacobi eigenbasis of
    (Ktilde, M).  No transform, no special basis, no closed form.

Route B (the structured factorization of Sections 5 and 6)
    V_reg in the special basis (eq:special_basis_dirichlet) written on the
    B-spline basis; U = [sin(x_i alpha_j)] (Table 1, D = {0,1}); Dt =
    diag(U^T V_reg^T M V_reg U)^{1/2} (end of Section 6); L_reg =
    |F_j|^2_H1 / ||F_j||^2_L2 (eq:Lambda reg2) by quadrature of F_j' and F_j,
    F_j = the spline with coefficients V_reg U e_j; V_out = M^{-1} W with W an orthonormal
    basis of range(V_reg)'s Euclidean complement; (L_out, Q_out) by Jacobi on
    the out pencil (eq:eigendecomposition_out).

Accuracy of the two routes.  Both are FP64.  Route A diagonalizes the full
projected pencil with Cholesky + Jacobi, whose eigenvalues carry absolute
errors of order eps * ||L^{-1} Ktilde L^{-T}|| ~ eps * n^2; the small
eigenvalues, which dominate P^{-1} r, therefore lose relative accuracy as n
grows (A and B differ by ~7e-12 at n = 192).  Route B's regular eigenvalues
are the seminorm quotients of exactly known modes, integrated from F_j' (no
cancellation of O(n^2) terms), and keep their relative accuracy, so it is the
reference for comparisons at large n; the two routes are checked against each
other (and against brute force) at small n.

Application (eq:preconditioner, eq:exact_diagonalization)
    z = (Qt x .. x Qt) (sum_k Lt_k)^{-1} (Qt^T x .. x Qt^T) r, with Qt^T
    applied first (the order the inverse requires), by explicit dense
    mode products on arrays stored with direction 1 fastest.
"""

from __future__ import annotations

import numpy as np

from . import bspline, eig


# ---------------------------------------------------------------------------
# Dimensions (eq:reg_space_dim, D = {0,1}) and nodes (eq:nodes, eq:delta)
# ---------------------------------------------------------------------------

def dims(n: int, p: int):
    m = n + p - 2
    n_reg = n - 1 if p % 2 else n
    n_out = p - 1 if p % 2 else p - 2
    return m, n_reg, n_out


def node(i, n: int, p: int):
    """x_i = i h (p odd), (i - 1/2) h (p even), eq:nodes."""
    h = 1.0 / n
    return i * h if p % 2 else (i - 0.5) * h


def delta_p(p: int) -> int:
    return 0 if p % 2 else 1


# ---------------------------------------------------------------------------
# Route A: splitting from the derivative conditions
# ---------------------------------------------------------------------------

def constraint_rows(n: int, p: int) -> np.ndarray:
    """E: rows d^{2k}/dx^{2k} of the reduced basis at x=0 and x=1,
    k = 1..floor((p-1)/2) (eq:reg_space with D = {0,1}); rows normalised."""
    knots = bspline.open_knots(n, p)
    rows = []
    for x in (0.0, 1.0):
        for k in range(1, (p - 1) // 2 + 1):
            r = bspline.derivative(knots, p, np.array([x]), 2 * k)[0, 1:-1]
            rows.append(r / np.linalg.norm(r))
    m = n + p - 2
    return np.array(rows).reshape(len(rows), m)


def factors_route_a(n: int, p: int):
    """(lam_t, Q_t, Ktilde, K, M) with Q_t^T M Q_t = I, Q_t^T Ktilde Q_t =
    diag(lam_t), lam_t ascending."""
    K, M = bspline.assemble_dirichlet(n, p)
    m = K.shape[0]
    E = constraint_rows(n, p)
    if E.shape[0] == 0:
        Kt = K.copy()
    else:
        Lm = eig.cholesky(M)
        Vout = eig.solve_upper_t(Lm, eig.solve_lower(Lm, E.T))   # M^{-1} E^T
        G = Vout.T @ M @ Vout
        Po = Vout @ np.linalg.solve(G, Vout.T @ M)
        Pr = np.eye(m) - Po
        Kt = Pr.T @ K @ Pr + Po.T @ K @ Po
        Kt = 0.5 * (Kt + Kt.T)
    lam, Q = eig.gen_eigh(Kt, M)
    return lam, Q, Kt, K, M


# ---------------------------------------------------------------------------
# Route B: special basis + sine transform (Sections 5, 6)
# ---------------------------------------------------------------------------

def cardinal_shift(i, n: int, p: int, x):
    """B~_i(x) = B~_p((x - x_i)/h), eq:Btilde (read with consistent units)."""
    return bspline.cardinal(p, (np.asarray(x) - node(i, n, p)) * n)


def special_basis_blocks(n: int, p: int):
    """Coefficients of the boundary functions of eq:special_basis_dirichlet on
    the B-spline basis: V0 (p-1 x floor(p/2)) on B_1..B_{p-1} and V1 on
    B_{m-p+2}..B_m.  Each boundary function lives on [0, ph] (resp.
    [1-ph, 1]), where only those p-1 reduced B-splines are active, so the
    coefficients follow from a collocation least-squares fit (exact up to
    rounding)."""
    knots = bspline.open_knots(n, p)
    m, n_reg, _ = dims(n, p)
    h = 1.0 / n
    half = p // 2
    dp = delta_p(p)
    # left end: Bhat_i = B~_i - B~_{dp - i}, i = 1..floor(p/2)
    xs = (np.arange(1, 4 * p + 1) - 0.5) / (4 * p) * (p * h)
    Bl = bspline.basis(knots, p, xs)[:, 1:p]
    V0 = np.zeros((p - 1, half))
    for c, i in enumerate(range(1, half + 1)):
        f = cardinal_shift(i, n, p, xs) - cardinal_shift(dp - i, n, p, xs)
        V0[:, c] = np.linalg.lstsq(Bl, f, rcond=None)[0]
    # right end: Bhat_i = B~_i - B~_{n + n_reg + 1 - i},
    # i = n_reg - floor(p/2) + 1 .. n_reg
    xr = 1.0 - xs[::-1]
    nb = n + p
    Br = bspline.basis(knots, p, xr)[:, nb - p:nb - 1]
    V1 = np.zeros((p - 1, half))
    for c, i in enumerate(range(n_reg - half + 1, n_reg + 1)):
        f = cardinal_shift(i, n, p, xr) - cardinal_shift(n + n_reg + 1 - i, n, p, xr)
        V1[:, c] = np.linalg.lstsq(Br, f, rcond=None)[0]
    return V0, V1


def special_vreg(n: int, p: int) -> np.ndarray:
    """V_reg (m x n_reg) for the special basis: blkdiag(V0, I_{n-p}, V1)
    (block structure of Section 4 with the basis of Section 6)."""
    m, n_reg, _ = dims(n, p)
    V0, V1 = special_basis_blocks(n, p)
    half = p // 2
    V = np.zeros((m, n_reg))
    V[:p - 1, :half] = V0
    V[p - 1:m - p + 1, half:n_reg - half] = np.eye(n - p)
    V[m - p + 1:, n_reg - half:] = V1
    return V


def sine_matrix(n: int, p: int) -> np.ndarray:
    """U_reg of Table 1 for D = {0,1}: U_ij = sin(x_i alpha_j), alpha_j = j pi,
    i, j = 1..n_reg (DST-I for odd p, DST-III / its transpose DST-II for even
    p), with unit weight in every column."""
    _, n_reg, _ = dims(n, p)
    i = np.arange(1, n_reg + 1)
    x = node(i, n, p)
    a = np.arange(1, n_reg + 1) * np.pi
    return np.sin(np.outer(x, a))


def mode_seminorms(n: int, p: int, C: np.ndarray):
    """|F|^2_H1 and ||F||^2_L2 of the splines F = sum_i C[i, j] B_i (reduced
    basis, one column per function), by Gauss-Legendre quadrature with p+1
    points per element, which is exact for both integrands (degree 2p-2 and
    2p).  F' is evaluated from the B-spline derivatives at the quadrature
    points and squared there, so no large terms cancel in the integral (the
    bilinear form C^T K C sums terms of size ~ n^2 |C|^2 into a result of size
    ~ |C|^2 for the smoothest modes)."""
    knots = bspline.open_knots(n, p)
    gx, gw = np.polynomial.legendre.leggauss(p + 1)
    e = np.arange(n)
    xq = ((e[:, None] + 0.5) + 0.5 * gx[None, :]).ravel() / n
    wq = np.tile(0.5 * gw / n, n)
    F = bspline.basis(knots, p, xq)[:, 1:-1] @ C
    dF = bspline.derivative(knots, p, xq, 1)[:, 1:-1] @ C
    return wq @ dF ** 2, wq @ F ** 2


def factors_route_b(n: int, p: int):
    """Structured factors: dict with V_reg, U, Dt, lam_reg, V_out, Q_out,
    lam_out, Qt (= [V_reg U Dt^{-1}, V_out Q_out]) and lam_t."""
    K, M = bspline.assemble_dirichlet(n, p)
    m, n_reg, n_out = dims(n, p)
    Vreg = special_vreg(n, p)
    U = sine_matrix(n, p)
    VU = Vreg @ U
    Dt2 = np.einsum("ij,ij->j", VU, M @ VU)
    h1, l2 = mode_seminorms(n, p, VU)
    lam_reg = h1 / l2
    Dt = np.sqrt(Dt2)
    Qreg_cols = VU / Dt
    if n_out:
        # orthonormal basis of the Euclidean complement of range(V_reg)
        Uc, S, _ = np.linalg.svd(Vreg, full_matrices=True)
        W = Uc[:, n_reg:]
        Lm = eig.cholesky(M)
        Vout = eig.solve_upper_t(Lm, eig.solve_lower(Lm, W))
        lam_out, Qout = eig.gen_eigh(Vout.T @ K @ Vout, Vout.T @ M @ Vout)
        Qt = np.hstack([Qreg_cols, Vout @ Qout])
        lam_t = np.concatenate([lam_reg, lam_out])
    else:
        Vout = np.zeros((m, 0))
        Qout = np.zeros((0, 0))
        lam_out = np.zeros(0)
        Qt = Qreg_cols
        lam_t = lam_reg
    return dict(K=K, M=M, V_reg=Vreg, U=U, Dt=Dt, lam_reg=lam_reg, V_out=Vout,
                Q_out=Qout, lam_out=lam_out, Qt=Qt, lam_t=lam_t)


def ktilde_from(Qt: np.ndarray, lam_t: np.ndarray) -> np.ndarray:
    """Ktilde = Qt^{-T} diag(lam_t) Qt^{-1} (Proposition 1)."""
    Qi = np.linalg.inv(Qt)
    return Qi.T @ np.diag(lam_t) @ Qi


# ---------------------------------------------------------------------------
# FD (Section 3): exact eigenbasis of the 1-D pencil (K, M)
# ---------------------------------------------------------------------------

def factors_fd(n: int, p: int):
    K, M = bspline.assemble_dirichlet(n, p)
    lam, Q = eig.gen_eigh(K, M)
    return lam, Q, K, M


# ---------------------------------------------------------------------------
# Kronecker applications on arrays of shape (..., m_d, ..., m_1)
# ---------------------------------------------------------------------------

def mode_product(X: np.ndarray, A: np.ndarray, direction: int, d: int) -> np.ndarray:
    """Apply the matrix A along direction `direction` (1-based; direction 1
    is the fastest, i.e. the last array axis) of the d-dimensional tensor X
    (leading batch axes allowed): Y[.., j, ..] = sum_l A[j, l] X[.., l, ..]."""
    ax = X.ndim - direction
    Xm = np.moveaxis(X, ax, -1)
    Y = Xm @ A.T
    return np.moveaxis(Y, -1, ax)


def kron_diag_apply(X, Qs, lams, d: int):
    """(Q_d x .. x Q_1) (sum_k lam_k)^{-1} (Q_d^T x .. x Q_1^T) X."""
    Y = X
    for k in range(1, d + 1):
        Y = mode_product(Y, Qs[k - 1].T, k, d)
    denom = 0.0
    for k in range(1, d + 1):
        shape = [1] * d
        shape[d - k] = len(lams[k - 1])
        denom = denom + lams[k - 1].reshape(shape)
    Y = Y / denom
    for k in range(1, d + 1):
        Y = mode_product(Y, Qs[k - 1], k, d)
    return Y


def kron_matvec(X, Ks, Ms, d: int):
    """Ahat X with Ahat = sum_k M_d x .. x K_k x .. x M_1 (eq:system_matrix,
    its d-term analogue), by mode products."""
    Y = np.zeros_like(X)
    for k in range(1, d + 1):
        T = X
        for j in range(1, d + 1):
            T = mode_product(T, Ks[j - 1] if j == k else Ms[j - 1], j, d)
        Y = Y + T
    return Y


class Preconditioner:
    """z = P^{-1} r for d dimensions, all directions with the same (n, p).

    kind = "iffd_a" (route A), "iffd_b" (route B) or "fd" (exact FD)."""

    def __init__(self, d: int, n: int, p: int, kind: str = "iffd_a"):
        self.d, self.n, self.p, self.kind = d, n, p, kind
        if kind == "iffd_a":
            lam, Q, Kt, K, M = factors_route_a(n, p)
        elif kind == "iffd_b":
            f = factors_route_b(n, p)
            lam, Q, K, M = f["lam_t"], f["Qt"], f["K"], f["M"]
            Kt = ktilde_from(Q, lam)
        elif kind == "fd":
            lam, Q, K, M = factors_fd(n, p)
            Kt = K
        else:
            raise ValueError(kind)
        self.lam, self.Q, self.Kt, self.K, self.M = lam, Q, Kt, K, M
        self.m = K.shape[0]

    def apply(self, R: np.ndarray) -> np.ndarray:
        d = self.d
        return kron_diag_apply(R, [self.Q] * d, [self.lam] * d, d)

    def matvec(self, X: np.ndarray) -> np.ndarray:
        d = self.d
        return kron_matvec(X, [self.K] * d, [self.M] * d, d)
