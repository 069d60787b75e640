"""The IFFD preconditioner with a Dirichlet set D_k per direction (D_k a
subset of {0, 1}: Dirichlet, Neumann or mixed conditions) and its own (n_k,
p_k) per direction.

Test infrastructure only (see the package docstring).  Shares no code with
the HIP implementation.

Per direction (Section 2, Section 4 "Other boundary conditions", Section 6):
    S_{p,h,D}   splines of degree p on n uniform elements that vanish on D:
                the B-spline B_0 is dropped when 0 is in D, the last one when
                1 is in D, so m = n + p - |D|.
    S^reg       (eq:reg_space) even derivatives 2, 4, .. <= p-1 vanish at the
                ends in D, odd derivatives 1, 3, .. <= p-1 at the other ends
                (reading of the odd-order range, see DESIGN); dims from
                eq:reg_space_dim.
    S^out       its L2-orthogonal complement.
Route A (definition): Ktilde = Pr^T K Pr + Po^T K Po from the constraint rows,
Jacobi eigenbasis of (Ktilde, M).  Route B (structure): the special basis of
eq:special_basis (B_L, B_I, B_R for each end type), U_reg = [sin(x_i alpha_j
+ beta)] of Table 1, Dt = diag(U^T V^T M V U)^{1/2}, Lambda_reg as seminorm
quotients (eq:Lambda reg2), V_out = M^{-1} W, Jacobi on the out pencil.
"""

from __future__ import annotations

import numpy as np

from . import bspline, eig
from . import iffd as _dir   # mode products and Kronecker applications only


def kept(n: int, p: int, D) -> np.ndarray:
    """Indices of the full B-spline basis (0 .. n+p-1) that span S_{p,h,D}."""
    idx = np.arange(n + p)
    if 0 in D:
        idx = idx[1:]
    if 1 in D:
        idx = idx[:-1]
    return idx


def assemble(n: int, p: int, D):
    K, M = bspline.assemble_full(n, p)
    k = kept(n, p, D)
    return K[np.ix_(k, k)].copy(), M[np.ix_(k, k)].copy()


def dims(n: int, p: int, D):
    """(m, n_reg, n_out), eq:reg_space_dim."""
    D = set(D)
    m = n + p - len(D)
    if p % 2 == 1 and D == {0, 1}:
        n_reg = n - 1
    elif p % 2 == 1 and not D:
        n_reg = n + 1
    else:
        n_reg = n
    return m, n_reg, m - n_reg


def constraint_rows(n: int, p: int, D) -> np.ndarray:
    """Rows of the derivative conditions of eq:reg_space on S_{p,h,D}: orders
    2, 4, .. <= p-1 at a Dirichlet end, 1, 3, .. <= p-1 at a Neumann end;
    each row normalised."""
    knots = bspline.open_knots(n, p)
    k = kept(n, p, D)
    rows = []
    for x in (0.0, 1.0):
        orders = range(2, p, 2) if x in D else range(1, p, 2)
        for r in orders:
            row = bspline.derivative(knots, p, np.array([x]), r)[0, k]
            rows.append(row / np.linalg.norm(row))
    return np.array(rows).reshape(len(rows), len(k))


def factors_route_a(n: int, p: int, D):
    K, M = assemble(n, p, D)
    m = K.shape[0]
    E = constraint_rows(n, p, D)
    if E.shape[0] == 0:
        Kt = K.copy()
    else:
        Lm = eig.cholesky(M)
        Vout = eig.solve_upper_t(Lm, eig.solve_lower(Lm, E.T))
        G = Vout.T @ M @ Vout
        Po = Vout @ np.linalg.solve(G, Vout.T @ M)
        Pr = np.eye(m) - Po
        Kt = Pr.T @ K @ Pr + Po.T @ K @ Po
        Kt = 0.5 * (Kt + Kt.T)
    lam, Q = eig.gen_eigh(Kt, M)
    return lam, Q, Kt, K, M


# ---- Table 1: nodes, frequencies and phases --------------------------------

def table1(n: int, p: int, D):
    """(x_i (i = 1..n_reg), alpha_j (j = 1..n_reg), beta) of Table 1."""
    D = set(D)
    _, n_reg, _ = dims(n, p, D)
    i = np.arange(1, n_reg + 1, dtype=np.float64)
    h = 1.0 / n
    if p % 2 == 1:
        x = i * h if 0 in D else (i - 1) * h
    else:
        x = (i - 0.5) * h
    if D == {0, 1}:
        a, beta = i * np.pi, 0.0
    elif D == {0}:
        a, beta = (i - 0.5) * np.pi, 0.0
    elif D == {1}:
        a, beta = (i - 0.5) * np.pi, np.pi / 2
    else:
        a, beta = (i - 1) * np.pi, np.pi / 2
    return x, a, beta


def sine_matrix(n: int, p: int, D) -> np.ndarray:
    x, a, beta = table1(n, p, D)
    return np.sin(np.outer(x, a) + beta)


# ---- the special basis (Section 6, eq:Btilde, eq:special_basis) -------------

def cardinal_at(k, n: int, p: int, x):
    """Btilde_k(x) = B_p((x - c_k)/h), centred at c_k = k h (p odd) or
    (k - 1/2) h (p even) (eq:Btilde with consistent units)."""
    c = k / n if p % 2 else (k - 0.5) / n
    return bspline.cardinal(p, (np.asarray(x) - c) * n)


def special_functions(n: int, p: int, D):
    """The ordered basis B_L u B_I u B_R as a list of (sign, index) lists:
    each function is sum_s sign * Btilde_index.  For 1 not in D and p even
    the index range of B_R is read as n - p/2 + 1 .. n (p/2 functions)."""
    D = set(D)
    dp = 0 if p % 2 else 1
    L, R = [], []
    if 0 in D:
        L = [[(1, i), (-1, dp - i)] for i in range(1, p // 2 + 1)]
    elif p % 2 == 0:
        L = [[(1, i), (1, 1 - i)] for i in range(1, p // 2 + 1)]
    else:
        L = [[(1, 0)]] + [[(1, i), (1, -i)] for i in range(1, (p - 1) // 2 + 1)]
    I = [[(1, i)] for i in range(p // 2 + 1, n - (p + 1) // 2 + 1)]
    if 1 in D:
        R = [[(1, i), (-1, 2 * n + dp - i)] for i in range(n - (p - 1) // 2, n + dp)]
    elif p % 2 == 0:
        R = [[(1, i), (1, 2 * n + 1 - i)] for i in range(n - p // 2 + 1, n + 1)]
    else:
        R = [[(1, i), (1, 2 * n - i)] for i in range(n - (p - 1) // 2, n)] + [[(1, n)]]
    return L + I + R


def special_vreg(n: int, p: int, D) -> np.ndarray:
    """Coefficients (m x n_reg) of the special basis functions, restricted to
    [0, 1], on the basis of S_{p,h,D}: least-squares collocation on dense
    points (exact up to rounding, the functions lie in the space)."""
    knots = bspline.open_knots(n, p)
    k = kept(n, p, D)
    xs = (np.arange(8 * (n + p)) + 0.5) / (8 * (n + p))
    B = bspline.basis(knots, p, xs)[:, k]
    funcs = special_functions(n, p, D)
    F = np.zeros((len(xs), len(funcs)))
    for c, terms in enumerate(funcs):
        for sgn, idx in terms:
            F[:, c] += sgn * cardinal_at(idx, n, p, xs)
    V, *_ = np.linalg.lstsq(B, F, rcond=None)
    return V


def factors_route_b(n: int, p: int, D):
    K, M = assemble(n, p, D)
    m, n_reg, n_out = dims(n, p, D)
    V = special_vreg(n, p, D)
    assert V.shape == (m, n_reg), (V.shape, m, n_reg)
    U = sine_matrix(n, p, D)
    VU = V @ U
    Dt2 = np.einsum("ij,ij->j", VU, M @ VU)
    # |F_j|^2_H1 / ||F_j||^2_L2 by quadrature on the full basis
    knots = bspline.open_knots(n, p)
    kk = kept(n, p, D)
    gx, gw = np.polynomial.legendre.leggauss(p + 1)
    e = np.arange(n)
    xq = ((e[:, None] + 0.5) + 0.5 * gx[None, :]).ravel() / n
    wq = np.tile(0.5 * gw / n, n)
    F = bspline.basis(knots, p, xq)[:, kk] @ VU
    dF = bspline.derivative(knots, p, xq, 1)[:, kk] @ VU
    lam_reg = (wq @ dF ** 2) / (wq @ F ** 2)
    Dt = np.sqrt(Dt2)
    Qreg = VU / Dt
    if n_out:
        Uc, _, _ = np.linalg.svd(V, full_matrices=True)
        W = Uc[:, n_reg:]
        Lm = eig.cholesky(M)
        Vout = eig.solve_upper_t(Lm, eig.solve_lower(Lm, W))
        lam_out, Qout = eig.gen_eigh(Vout.T @ K @ Vout, Vout.T @ M @ Vout)
        Qt = np.hstack([Qreg, Vout @ Qout])
        lam_t = np.concatenate([lam_reg, lam_out])
    else:
        Vout, Qout, lam_out = np.zeros((m, 0)), np.zeros((0, 0)), np.zeros(0)
        Qt, lam_t = Qreg, lam_reg
    return dict(K=K, M=M, V_reg=V, U=U, Dt=Dt, lam_reg=lam_reg, V_out=Vout, Q_out=Qout,
                lam_out=lam_out, Qt=Qt, lam_t=lam_t)


# ---- a generic basis of S^reg (eq:reg_eigenvectors) --------------------------

def end_block_sizes(n: int, p: int, D):
    """(cl, cr): the number of special-basis functions of B_L and B_R (the
    counts of special_functions)."""
    D = set(D)
    cl = p // 2 if (0 in D or p % 2 == 0) else (p + 1) // 2
    cr = p // 2 if (1 in D or p % 2 == 0) else (p + 1) // 2
    return cl, cr


def generic_vreg(n: int, p: int, D):
    """A basis of S^reg other than the special one: each end block of the
    special basis (its cl or cr functions, written on the B-splines they
    touch) replaced by the orthonormal columns Q of its QR factorization,
    diagonal of R positive; the interior B-splines are kept.  Returns
    (V_generic, V_special, (rl, cl, rr, cr))."""
    V = special_vreg(n, p, D)
    m, n_reg = V.shape
    cl, cr = end_block_sizes(n, p, D)
    tol = 1e-12 * np.abs(V).max()
    rl = 1 + max([r for r in range(m) if np.abs(V[r, :cl]).max(initial=0.0) > tol], default=-1)
    rr = m - min([r for r in range(m) if np.abs(V[r, n_reg - cr:]).max(initial=0.0) > tol],
                 default=m)
    Vg = V.copy()

    def orth(A):
        Q, R = np.linalg.qr(A)
        return Q * np.sign(np.diag(R))

    if cl:
        Vg[:rl, :cl] = orth(V[:rl, :cl])
    if cr:
        Vg[m - rr:, n_reg - cr:] = orth(V[m - rr:, n_reg - cr:])
    return Vg, V, (rl, cl, rr, cr)


def collocation(n: int, p: int, D, V) -> np.ndarray:
    """C_ij = psi_j(x_i): the basis psi (coefficients V on the B-splines of
    S_{p,h,D}) at the nodes x_i of Table 1 (the interpolation matrix of
    eq:reg_eigenvectors, whose C^{-1} interpolates)."""
    x, _, _ = table1(n, p, D)
    knots = bspline.open_knots(n, p)
    return bspline.basis(knots, p, x)[:, kept(n, p, D)] @ V


def factors_generic(n: int, p: int, D):
    """Q_reg = C^{-1} U D^{-1} (eq:reg_eigenvectors) in the generic basis:
    the columns of C^{-1} U are the coefficients of the interpolants F_j of
    sin(x alpha_j + beta) at the nodes; D_jj = ||F_j||_L2 (eq:Dreg2, the mass
    matrix of S^reg); Lambda_reg = D^{-1} U^T C^{-T} V^T K V C^{-1} U D^{-1}
    (eq:Lambda reg), whose diagonal is kept (the off-diagonal part vanishes,
    the F_j being the discrete eigenfunctions).  The outlier part is that of
    route B (S^out does not depend on the basis of S^reg)."""
    K, M = assemble(n, p, D)
    Vg, _, sizes = generic_vreg(n, p, D)
    U = sine_matrix(n, p, D)
    C = collocation(n, p, D, Vg)
    W = np.linalg.solve(C, U)
    VF = Vg @ W
    Dg = np.sqrt(np.einsum("ij,ij->j", VF, M @ VF))
    Qreg = W / Dg
    VQ = Vg @ Qreg
    Lfull = VQ.T @ K @ VQ
    lam_reg = np.diag(Lfull).copy()
    fb = factors_route_b(n, p, D)
    Vout, Qout, lam_out = fb["V_out"], fb["Q_out"], fb["lam_out"]
    Qt = np.hstack([VQ, Vout @ Qout]) if Vout.shape[1] else VQ
    lam_t = np.concatenate([lam_reg, lam_out])
    return dict(K=K, M=M, V_reg=Vg, C=C, U=U, W=W, D=Dg, Q_reg=Qreg, Lambda_full=Lfull,
                lam_reg=lam_reg, Qt=Qt, lam_t=lam_t, sizes=sizes)


class GeneralPreconditioner:
    """z = P^{-1} r on [0,1]^d with per-direction specs (n_k, p_k, D_k),
    direction 1 first (the fastest index).  kind: "iffd_a", "iffd_b", "fd",
    "iffd_generic" (route B's operator through the generic basis of
    eq:reg_eigenvectors)."""

    def __init__(self, specs, kind: str = "iffd_b"):
        self.specs = [(int(n), int(p), frozenset(D)) for n, p, D in specs]
        self.d = len(self.specs)
        self.kind = kind
        self.Q, self.lam, self.K, self.M = [], [], [], []
        for n, p, D in self.specs:
            if kind == "iffd_a":
                lam, Q, _, K, M = factors_route_a(n, p, D)
            elif kind == "iffd_b":
                f = factors_route_b(n, p, D)
                lam, Q, K, M = f["lam_t"], f["Qt"], f["K"], f["M"]
            elif kind == "iffd_generic":
                f = factors_generic(n, p, D)
                lam, Q, K, M = f["lam_t"], f["Qt"], f["K"], f["M"]
            elif kind == "fd":
                K, M = assemble(n, p, D)
                lam, Q = eig.gen_eigh(K, M)
            else:
                raise ValueError(kind)
            self.Q.append(Q)
            self.lam.append(lam)
            self.K.append(K)
            self.M.append(M)
        self.shape = tuple(K.shape[0] for K in reversed(self.K))   # (m_d, .., m_1)

    def apply(self, R):
        return _dir.kron_diag_apply(R, self.Q, self.lam, self.d)

    def matvec(self, X):
        return _dir.kron_matvec(X, self.K, self.M, self.d)
