"""IFFD with reduced regularity at an interior knot (Remark
rmk:reduced_regularity, eq:reg_space2), per direction.

Test infrastructure only (see the package docstring).  Shares no code with
the HIP implementation.

Per direction: the uniform knot vector of degree p on n elements with the
interior breakpoint xi* = k/n repeated `mult` times (1 <= mult <= p), so the
spline space S' is C^{p - mult} at xi* and has n + p + mult - 1 B-splines
before the Dirichlet ends drop theirs (Section 2).
    S^reg   (eq:reg_space2) the functions of S' that are C^{p-1} everywhere
            and satisfy the end conditions of eq:reg_space: the regular space
            of the maximally smooth space, unchanged by the repeated knot.
    S^out   its L2-orthogonal complement in S': one dimension more per extra
            copy of the knot.
Route A (definition): the constraint rows are those of the ends (eq:reg_space,
as in oracle.general) plus the jumps of the derivatives of orders
p - mult + 1 .. p - 1 at xi*; Ktilde = Pr^T K Pr + Po^T K Po, Jacobi
eigenbasis of (Ktilde, M).
Route B (structure): the special basis functions of eq:special_basis written
on the B-splines of S' by collocation (they are C^{p-1} splines on the
uniform knots, so they lie in S'), U of Table 1, Dt = diag(U^T V^T M V U)^{1/2},
Lambda_reg as seminorm quotients (eq:Lambda reg2), V_out = M^{-1} W with W
spanning the Euclidean complement of range(V_reg), Jacobi on the out pencil.
"""

from __future__ import annotations

import numpy as np

from . import bspline, eig
from . import general as G
from . import iffd as _dir   # mode products and Kronecker applications only


def knots(n: int, p: int, k: int, mult: int) -> np.ndarray:
    """The p-open uniform knots with the breakpoint k/n repeated mult times."""
    assert 1 <= mult <= p and 0 < k < n
    return np.sort(np.concatenate([bspline.open_knots(n, p), np.full(mult - 1, k / n)]))


def kept(nb: int, D) -> np.ndarray:
    idx = np.arange(nb)
    if 0 in D:
        idx = idx[1:]
    if 1 in D:
        idx = idx[:-1]
    return idx


def assemble(n: int, p: int, D, k: int, mult: int):
    """K and M of S'_{D} by Gauss-Legendre with p+1 points per element (exact)."""
    kn = knots(n, p, k, mult)
    nb = len(kn) - p - 1
    gx, gw = np.polynomial.legendre.leggauss(p + 1)
    K = np.zeros((nb, nb))
    M = np.zeros((nb, nb))
    for e in range(n):
        a, b = e / n, (e + 1) / n
        xq = 0.5 * (a + b) + 0.5 * (b - a) * gx
        wq = 0.5 * (b - a) * gw
        B = bspline.basis(kn, p, xq)
        dB = bspline.derivative(kn, p, xq, 1)
        M += (B * wq[:, None]).T @ B
        K += (dB * wq[:, None]).T @ dB
    kk = kept(nb, D)
    return K[np.ix_(kk, kk)].copy(), M[np.ix_(kk, kk)].copy()


def dims(n: int, p: int, D, mult: int):
    """(m, n_reg, n_out): n_reg as for the maximally smooth space
    (eq:reg_space_dim), n_out larger by mult - 1."""
    _, n_reg, _ = G.dims(n, p, D)
    m = n + p + mult - 1 - len(set(D))
    return m, n_reg, m - n_reg


def constraint_rows(n: int, p: int, D, k: int, mult: int) -> np.ndarray:
    kn = knots(n, p, k, mult)
    kk = kept(len(kn) - p - 1, D)
    rows = []
    for x in (0.0, 1.0):
        orders = range(2, p, 2) if x in D else range(1, p, 2)
        for r in orders:
            row = bspline.derivative(kn, p, np.array([x]), r)[0, kk]
            rows.append(row / np.linalg.norm(row))
    xs = np.array([k / n])
    for q in range(p - mult + 1, p):
        row = (bspline.derivative(kn, p, xs, q)[0, kk]
               - bspline.derivative(kn, p, xs, q, left=True)[0, kk])
        rows.append(row / np.linalg.norm(row))
    return np.array(rows).reshape(len(rows), len(kk))


def factors_route_a(n: int, p: int, D, k: int, mult: int):
    K, M = assemble(n, p, D, k, mult)
    m = K.shape[0]
    E = constraint_rows(n, p, D, k, mult)
    if E.shape[0] == 0:
        Kt = K.copy()
    else:
        Lm = eig.cholesky(M)
        Vout = eig.solve_upper_t(Lm, eig.solve_lower(Lm, E.T))
        Gm = Vout.T @ M @ Vout
        Po = Vout @ np.linalg.solve(Gm, Vout.T @ M)
        Pr = np.eye(m) - Po
        Kt = Pr.T @ K @ Pr + Po.T @ K @ Po
        Kt = 0.5 * (Kt + Kt.T)
    lam, Q = eig.gen_eigh(Kt, M)
    return lam, Q, K, M


def special_vreg(n: int, p: int, D, k: int, mult: int) -> np.ndarray:
    """Coefficients (m x n_reg) of the special basis functions on the
    B-splines of S'_D: least-squares collocation on dense points."""
    kn = knots(n, p, k, mult)
    kk = kept(len(kn) - p - 1, D)
    xs = (np.arange(8 * (n + p)) + 0.5) / (8 * (n + p))
    B = bspline.basis(kn, p, xs)[:, kk]
    funcs = G.special_functions(n, p, D)
    F = np.zeros((len(xs), len(funcs)))
    for c, terms in enumerate(funcs):
        for sgn, idx in terms:
            F[:, c] += sgn * G.cardinal_at(idx, n, p, xs)
    V, *_ = np.linalg.lstsq(B, F, rcond=None)
    return V


def factors_route_b(n: int, p: int, D, k: int, mult: int):
    K, M = assemble(n, p, D, k, mult)
    m, n_reg, n_out = dims(n, p, D, mult)
    V = special_vreg(n, p, D, k, mult)
    assert V.shape == (m, n_reg)
    U = G.sine_matrix(n, p, D)
    VU = V @ U
    Dt = np.sqrt(np.einsum("ij,ij->j", VU, M @ VU))
    kn = knots(n, p, k, mult)
    kk = kept(len(kn) - p - 1, D)
    gx, gw = np.polynomial.legendre.leggauss(p + 1)
    e = np.arange(n)
    xq = ((e[:, None] + 0.5) + 0.5 * gx[None, :]).ravel() / n
    wq = np.tile(0.5 * gw / n, n)
    F = bspline.basis(kn, p, xq)[:, kk] @ VU
    dF = bspline.derivative(kn, p, xq, 1)[:, kk] @ VU
    lam_reg = (wq @ dF ** 2) / (wq @ F ** 2)
    Qreg = VU / Dt
    Uc, _, _ = np.linalg.svd(V, full_matrices=True)
    W = Uc[:, n_reg:]
    Lm = eig.cholesky(M)
    Vout = eig.solve_upper_t(Lm, eig.solve_lower(Lm, W))
    lam_out, Qout = eig.gen_eigh(Vout.T @ K @ Vout, Vout.T @ M @ Vout)
    Qt = np.hstack([Qreg, Vout @ Qout])
    lam_t = np.concatenate([lam_reg, lam_out])
    return dict(K=K, M=M, V_reg=V, U=U, Dt=Dt, lam_reg=lam_reg, V_out=Vout, Q_out=Qout,
                lam_out=lam_out, Qt=Qt, lam_t=lam_t)


class ReducedPreconditioner:
    """z = P^{-1} r with per-direction specs (n_k, p_k, D_k, knot_k), knot_k
    None (maximal smoothness, oracle.general) or (k, mult); direction 1
    first.  kind: "iffd_a", "iffd_b", "fd"."""

    def __init__(self, specs, kind: str = "iffd_b"):
        self.specs = [(int(n), int(p), frozenset(D), None if kt is None else tuple(kt))
                      for n, p, D, kt in specs]
        self.d = len(self.specs)
        self.Q, self.lam, self.K, self.M = [], [], [], []
        for n, p, D, kt in self.specs:
            if kt is None:
                g = G.GeneralPreconditioner([(n, p, set(D))], kind)
                Q, lam, K, M = g.Q[0], g.lam[0], g.K[0], g.M[0]
            elif kind == "iffd_a":
                lam, Q, K, M = factors_route_a(n, p, D, *kt)
            elif kind == "iffd_b":
                f = factors_route_b(n, p, D, *kt)
                lam, Q, K, M = f["lam_t"], f["Qt"], f["K"], f["M"]
            elif kind == "fd":
                K, M = assemble(n, p, D, *kt)
                lam, Q = eig.gen_eigh(K, M)
            else:
                raise ValueError(kind)
            self.Q.append(Q)
            self.lam.append(lam)
            self.K.append(K)
            self.M.append(M)
        self.shape = tuple(K.shape[0] for K in reversed(self.K))

    def apply(self, R):
        return _dir.kron_diag_apply(R, self.Q, self.lam, self.d)

    def matvec(self, X):
        return _dir.kron_matvec(X, self.K, self.M, self.d)
