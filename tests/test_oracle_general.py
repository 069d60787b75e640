"""Pins for oracle.general (Dirichlet, Neumann and mixed conditions per
direction): the dimension table eq:reg_space_dim, the derivative conditions
of eq:reg_space on the special basis, Theorems 3 and 5 for every column of
Table 1 (both parities), route A (definition) = route B (special basis and
Table 1 transforms) = brute force, the p = 1 and (p = 2, D = {0,1}) special
cases, and the Table 3 iteration counts."""

import json
import os

import numpy as np
import pytest

from oracle import bspline, krylov
from oracle import general as G
from oracle import iffd as O

CASES = [frozenset(s) for s in ({0, 1}, {0}, {1}, set())]
HERE = os.path.dirname(os.path.abspath(__file__))


def dims_typed(n, p, D):
    """eq:reg_space_dim, typed in from the paper: n_reg = n-1 (p odd, D =
    {0,1}), n+1 (p odd, D = {}), n otherwise; n_out = p-2 (p even, D = {0,1}),
    p (p even, D = {}), p-1 otherwise."""
    D = set(D)
    if p % 2:
        n_reg = n - 1 if D == {0, 1} else (n + 1 if not D else n)
    else:
        n_reg = n
    if p % 2 == 0 and D == {0, 1}:
        n_out = p - 2
    elif p % 2 == 0 and not D:
        n_out = p
    else:
        n_out = p - 1
    return n_reg, n_out


def symbol(q, kmax, t):
    return sum(bspline.cardinal(q, float(k)) * np.cos(k * t) for k in range(-kmax, kmax + 1))


@pytest.mark.parametrize("D", CASES, ids=lambda D: "D" + "".join(map(str, sorted(D))))
@pytest.mark.parametrize("p", range(1, 9))
def test_dimensions_constraints_and_theorems(p, D):
    n = 2 * p + 8
    m, n_reg, n_out = G.dims(n, p, D)
    assert (n_reg, n_out) == dims_typed(n, p, D) and m == n + p - len(D)
    fb = G.factors_route_b(n, p, D)
    K, M, V, U = fb["K"], fb["M"], fb["V_reg"], fb["U"]
    assert V.shape == (m, n_reg) and np.linalg.matrix_rank(V) == n_reg
    E = G.constraint_rows(n, p, D)
    assert E.shape == (n_out, m)
    if n_out:
        assert np.abs(E @ V).max() < 1e-12
        Vo = fb["V_out"]
        assert np.abs(V.T @ M @ Vo).max() < 1e-12 * np.abs(V).max() * np.abs(M).max() * np.abs(Vo).max() * m
    # Theorem 3: U^T M_reg U and U^T K_reg U are diagonal
    for A in (V.T @ M @ V, V.T @ K @ V):
        Dg = U.T @ A @ U
        off = Dg - np.diag(Dg.diagonal())
        assert np.abs(off).max() <= 1e-12 * np.abs(Dg.diagonal()).max()
    # Theorem 5: C_reg U = U Theta, C_ij = Bhat_j(x_i) at the nodes of Table 1
    x, a, _ = G.table1(n, p, D)
    C = bspline.basis(bspline.open_knots(n, p), p, x)[:, G.kept(n, p, D)] @ V
    np.testing.assert_allclose(C @ U, U * symbol(p, p // 2, a / n), atol=1e-12)


@pytest.mark.parametrize("D", CASES, ids=lambda D: "D" + "".join(map(str, sorted(D))))
@pytest.mark.parametrize("p", range(1, 9))
def test_route_a_equals_route_b(p, D):
    n = 2 * p + 8
    lamA, QA, KtA, K, M = G.factors_route_a(n, p, D)
    fb = G.factors_route_b(n, p, D)
    np.testing.assert_allclose(np.sort(fb["lam_t"]), lamA, rtol=1e-10, atol=1e-12 * lamA.max())
    np.testing.assert_allclose(fb["Qt"].T @ M @ fb["Qt"], np.eye(len(lamA)), atol=1e-11)
    assert lamA.min() > -1e-10 * lamA.max()
    if not D:   # pure Neumann: the constants are the kernel (alpha_1 = 0)
        assert abs(lamA[0]) < 1e-9 * lamA.max() and abs(fb["lam_reg"][0]) < 1e-12 * lamA.max()
    else:
        assert lamA[0] > 0


def test_dirichlet_case_is_the_symmetric_oracle():
    """D = {0, 1} reproduces the Dirichlet-only oracle (oracle.iffd)."""
    for p in (2, 3, 4, 7):
        n = 16
        a = G.factors_route_b(n, p, {0, 1})
        b = O.factors_route_b(n, p)
        np.testing.assert_allclose(a["lam_t"], b["lam_t"], rtol=1e-12)
        np.testing.assert_allclose(a["V_reg"], b["V_reg"], atol=1e-12)


@pytest.mark.parametrize("specs", [
    [(6, 3, {0}), (5, 2, {1})],
    [(6, 4, set()), (7, 3, {0})],
    [(4, 2, {0}), (4, 3, {1}), (3, 2, {0, 1})],
    [(5, 5, {1}), (4, 2, set()), (4, 3, {0})]])
def test_brute_force_mixed(specs):
    """P^{-1} r from routes A and B against the dense solve with the
    assembled P = sum_k M x .. x Ktilde_k x .. x M (Proposition 1) on tiny
    anisotropic problems; P is SPD when some direction has a Dirichlet end."""
    pa = G.GeneralPreconditioner(specs, "iffd_a")
    pb = G.GeneralPreconditioner(specs, "iffd_b")
    d = len(specs)
    r = np.random.default_rng(len(specs)).uniform(-1, 1, pa.shape)
    Kts = []
    for n, p, D in pa.specs:
        Kts.append(G.factors_route_a(n, p, D)[2])
    # explicit Kronecker products, direction 1 fastest (the last factor)
    P = np.zeros((r.size, r.size))
    for k in range(d):
        T = np.ones((1, 1))
        for j in range(d - 1, -1, -1):
            T = np.kron(T, Kts[j] if j == k else pa.M[j])
        P += T
    assert np.all(np.linalg.eigvalsh(P) > 0)
    z = np.linalg.solve(P, r.ravel()).reshape(r.shape)
    for pre in (pa, pb):
        assert np.linalg.norm(pre.apply(r) - z) <= 1e-11 * np.linalg.norm(z)


@pytest.mark.parametrize("D", CASES, ids=lambda D: "D" + "".join(map(str, sorted(D))))
def test_p1_is_fd(D):
    """p = 1: S^reg = S, the preconditioner is the exact inverse (with a
    Dirichlet direction beside it so the 2D operator is nonsingular)."""
    specs = [(12, 1, D), (10, 1, {0})]
    pb = G.GeneralPreconditioner(specs, "iffd_b")
    fd = G.GeneralPreconditioner(specs, "fd")
    r = np.random.default_rng(3).uniform(-1, 1, pb.shape)
    assert np.linalg.norm(pb.apply(r) - fd.apply(r)) <= 1e-12 * np.linalg.norm(fd.apply(r))


def test_table3_counts_n64():
    """Table 3, n = 64 (3D mixed: D = {0}, {1}, {} in directions 1, 2, 3): the
    oracle's PCG counts for p = 2..5 within +-1 of the printed 7, 7, 7, 6."""
    g = json.load(open(os.path.join(HERE, "golden", "table3_cube.json")))
    printed = g["iterations"][g["n"].index(64)]
    for p, it_p in zip(g["p"], printed):
        specs = [(64, p, {0}), (64, p, {1}), (64, p, set())]
        pre = G.GeneralPreconditioner(specs, "iffd_b")
        f = np.random.default_rng(1).uniform(-1, 1, pre.shape)
        _, it, conv, *_ = krylov.pcg(pre.matvec, pre.apply, f, tol=1e-8)
        assert conv and abs(it - it_p) <= 1, (p, it, it_p)


@pytest.mark.parametrize("D", CASES, ids=lambda D: "D" + "".join(map(str, sorted(D))))
@pytest.mark.parametrize("p", range(1, 9))
def test_generic_basis_route(p, D):
    """eq:reg_eigenvectors with two bases of S^reg.  The special basis: its
    collocation matrix C_s (psi_j at the nodes x_i of Table 1) has the columns
    of U as eigenvectors (C_s U = U Theta, Theta > 0).  The generic basis (end
    blocks orthonormalized): U does not diagonalize C, but Q_reg = C^{-1} U
    D^{-1} gives M-orthonormal eigenvectors (eq:Lambda reg is diagonal) with
    the same eigenvalues as route B, and the same P^{-1} r."""
    n = 2 * p + 8
    f = G.factors_generic(n, p, D)
    fb = G.factors_route_b(n, p, D)
    U = f["U"]
    Vs = G.special_vreg(n, p, D)
    T = np.linalg.solve(U, G.collocation(n, p, D, Vs) @ U)
    theta = np.diag(T)
    assert np.abs(T - np.diag(theta)).max() < 1e-12 and theta.min() > 0
    Tg = np.linalg.solve(U, f["C"] @ U)
    cl, cr = G.end_block_sizes(n, p, D)
    if max(cl, cr) >= 2 or (D != {0, 1} and p >= 2):
        assert np.abs(Tg - np.diag(np.diag(Tg))).max() > 1e-3   # the solve is needed
    Vg = f["V_reg"]
    VQ = Vg @ f["Q_reg"]
    assert np.abs(VQ.T @ fb["M"] @ VQ - np.eye(VQ.shape[1])).max() < 1e-12
    Lf = f["Lambda_full"]
    assert np.abs(Lf - np.diag(np.diag(Lf))).max() < 1e-12 * np.abs(Lf).max()
    assert np.abs(f["lam_reg"] - fb["lam_reg"]).max() <= 1e-12 * fb["lam_reg"].max()
    # the same preconditioner (shifted by the identity where D is empty: lambda_0 = 0)
    r = np.random.default_rng(p).standard_normal(f["Qt"].shape[0])
    za = f["Qt"] @ ((f["Qt"].T @ r) / (f["lam_t"] + 1.0))
    zb = fb["Qt"] @ ((fb["Qt"].T @ r) / (fb["lam_t"] + 1.0))
    assert np.abs(za - zb).max() <= 1e-12 * np.abs(zb).max()
