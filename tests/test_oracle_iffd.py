"""Pins for oracle.iffd: dimension counts, the splitting, Theorems 3 and 5,
the (corrected) Lemma 4 closed forms, route A = route B, brute force, the
p = 2 exactness, FD = direct solve, and the condition-number bound."""

import numpy as np
import pytest
import scipy.linalg

from oracle import brute, bspline, iffd, krylov


def dims_table(n, p):
    """eq:reg_space_dim for D = {0,1}, typed in from the paper."""
    return (n - 1 if p % 2 == 1 else n), (p - 1 if p % 2 == 1 else p - 2)


@pytest.mark.parametrize("p", range(1, 9))
def test_dimensions_and_constraints(p):
    n = 2 * p + 5
    m, n_reg, n_out = iffd.dims(n, p)
    assert (n_reg, n_out) == dims_table(n, p) and m == n_reg + n_out == n + p - 2
    E = iffd.constraint_rows(n, p)
    assert E.shape == (n_out, m)
    if n_out:
        assert np.linalg.matrix_rank(E) == n_out
    if p >= 2:
        V = iffd.special_vreg(n, p)
        assert V.shape == (m, n_reg) and np.linalg.matrix_rank(V) == n_reg
        # the special basis satisfies the derivative conditions of eq:reg_space
        if n_out:
            assert np.abs(E @ V).max() < 1e-10
        f = iffd.factors_route_b(n, p)
        K, M = f["K"], f["M"]
        if n_out:
            Vo = f["V_out"]
            scale = np.abs(V).max() * np.abs(M).max() * np.abs(Vo).max() * m
            assert np.abs(V.T @ M @ Vo).max() < 1e-13 * scale
            assert np.linalg.matrix_rank(np.hstack([V, f["V_out"]])) == m


@pytest.mark.parametrize("p", range(2, 9))
def test_special_basis_interior_is_bsplines(p):
    n = 3 * p + 2
    m, n_reg, _ = iffd.dims(n, p)
    knots = bspline.open_knots(n, p)
    x = np.linspace(0, 1, 601)
    B = bspline.basis(knots, p, x)
    half = p // 2
    for i in range(half + 1, n_reg - half + 1):
        l = i + (p - 1) // 2 if p % 2 else i + p // 2 - 1
        np.testing.assert_allclose(iffd.cardinal_shift(i, n, p, x), B[:, l], atol=1e-12)
    # and the boundary functions vanish at the Dirichlet ends
    V = iffd.special_vreg(n, p)
    assert np.abs(V[0, :]).max() > 0


@pytest.mark.parametrize("p", range(2, 9))
@pytest.mark.parametrize("n", [12, 17])
def test_theorem3_and_theorem5(p, n):
    if n <= p:
        pytest.skip("n > p assumed")
    f = iffd.factors_route_b(n, p)
    K, M, V, U = f["K"], f["M"], f["V_reg"], f["U"]
    for A in (V.T @ M @ V, V.T @ K @ V):
        D = U.T @ A @ U
        off = D - np.diag(D.diagonal())
        assert np.abs(off).max() <= 1e-12 * np.abs(D.diagonal()).max()
    # Theorem 5: C_reg U = U Theta, C_ij = Bhat_j(x_i)
    m, n_reg, _ = iffd.dims(n, p)
    knots = bspline.open_knots(n, p)
    xi = iffd.node(np.arange(1, n_reg + 1), n, p)
    C = bspline.basis(knots, p, xi)[:, 1:-1] @ V
    h = 1.0 / n
    th = np.zeros(n_reg)
    for k in range(-(p // 2), p // 2 + 1):
        th += bspline.cardinal(p, float(k)) * np.cos(k * h * np.arange(1, n_reg + 1) * np.pi)
    np.testing.assert_allclose(C @ U, U * th, atol=1e-12)


def symbol(q, kmax, theta):
    s = 0.0
    for k in range(-kmax, kmax + 1):
        s = s + bspline.cardinal(q, float(k)) * np.cos(k * theta)
    return s


@pytest.mark.parametrize("p", range(2, 9))
def test_lemma4_corrected_closed_forms(p):
    """Lemma 4 with the h-scaling read as in its proof (stiffness symbol
    (2 - 2cos)/h^2 times the degree 2p-1 symbol, mass symbol h * degree 2p+1
    symbol) and the special-basis normalisation Dt = D_reg Theta:
    lam_reg = (2-2cos t)/h^2 * sK/sM, Dt^2 = sM * ||q_j||^2 / (4n), where
    ||q_j||^2 = 2n except 4n for the alternating mode j = n (p even)."""
    n = 16
    h = 1.0 / n
    f = iffd.factors_route_b(n, p)
    _, n_reg, _ = iffd.dims(n, p)
    j = np.arange(1, n_reg + 1)
    t = j * np.pi * h
    sM = symbol(2 * p + 1, p, t)
    sK = symbol(2 * p - 1, p - 1, t)
    lam = (2 - 2 * np.cos(t)) / h ** 2 * sK / sM
    np.testing.assert_allclose(f["lam_reg"], lam, rtol=1e-12)
    qn = np.where(j == n, 4 * n, 2 * n)
    np.testing.assert_allclose(f["Dt"] ** 2, sM * qn / (4 * n), rtol=1e-12)


@pytest.mark.parametrize("n,p", [(256, 3), (192, 4)])
def test_regular_eigenvalues_keep_relative_accuracy_at_large_n(n, p):
    """Route B's smooth-mode eigenvalues (seminorm quotients integrated from
    F_j', eq:Lambda reg2) against Lemma 4's closed form with 2 - 2cos t written
    as 4 sin^2(t/2), which has no cancellation on smooth modes: 1e-14 on the
    first modes.  The FP64 quotient x^T K x / x^T M x of the same modes is off
    by eps * n^2 (4e-13 at n = 256), which this would catch."""
    h = 1.0 / n
    f = iffd.factors_route_b(n, p)
    j = np.arange(1, 9)
    t = j * np.pi * h
    lam = 4 * np.sin(t / 2) ** 2 / h ** 2 * symbol(2 * p - 1, p - 1, t) / symbol(2 * p + 1, p, t)
    np.testing.assert_allclose(f["lam_reg"][:8], lam, rtol=1e-14)


def test_p1_route_b_is_fd():
    """p = 1: S^reg = S (no outliers), the special basis is the B-spline basis
    and U diagonalizes K and M exactly, so route B is the FD inverse."""
    for d, n in ((2, 24), (3, 8)):
        fb = iffd.factors_route_b(n, 1)
        assert fb["V_out"].shape[1] == 0
        r = np.random.default_rng(d).uniform(-1, 1, (n - 1,) * d)
        zb = iffd.Preconditioner(d, n, 1, "iffd_b").apply(r)
        zf = iffd.Preconditioner(d, n, 1, "fd").apply(r)
        assert np.linalg.norm(zb - zf) <= 1e-13 * np.linalg.norm(zf)


@pytest.mark.parametrize("p", range(1, 9))
def test_route_a_equals_route_b(p):
    n = 2 * p + 6
    lamA, QA, KtA, K, M = iffd.factors_route_a(n, p)
    if p >= 2:
        fb = iffd.factors_route_b(n, p)
        np.testing.assert_allclose(np.sort(fb["lam_t"]), lamA, rtol=1e-11)
        np.testing.assert_allclose(fb["Qt"].T @ M @ fb["Qt"], np.eye(len(lamA)), atol=1e-12)
        for d in (2, 3):
            r = np.random.default_rng(p + d).uniform(-1, 1, (iffd.dims(n, p)[0],) * d)
            za = iffd.Preconditioner(d, n, p, "iffd_a").apply(r)
            zb = iffd.Preconditioner(d, n, p, "iffd_b").apply(r)
            assert np.linalg.norm(za - zb) <= 1e-11 * np.linalg.norm(za)
    np.testing.assert_allclose(QA.T @ KtA @ QA, np.diag(lamA), atol=1e-10 * lamA.max())
    assert lamA.min() > 0


@pytest.mark.parametrize("d,n,p", [(2, 6, 2), (2, 7, 3), (2, 8, 4), (2, 9, 5), (2, 10, 6),
                                   (2, 12, 8), (3, 4, 2), (3, 4, 3), (3, 5, 4)])
def test_brute_force(d, n, p):
    pre = iffd.Preconditioner(d, n, p, "iffd_a")
    fd = iffd.Preconditioner(d, n, p, "fd")
    m = pre.m
    A = brute.dense_system(pre.K, pre.M, d)
    P = brute.dense_preconditioner(pre.Kt, pre.M, d)
    np.linalg.cholesky(P)   # P is SPD
    r = np.random.default_rng(d * 100 + p).uniform(-1, 1, (m,) * d)
    z = pre.apply(r)
    zd = np.linalg.solve(P, r.reshape(-1)).reshape(r.shape)
    assert np.linalg.norm(z - zd) <= 1e-12 * np.linalg.norm(zd)
    # FD is a direct solver for Ahat (Section 3)
    zf = fd.apply(r)
    za = np.linalg.solve(A, r.reshape(-1)).reshape(r.shape)
    assert np.linalg.norm(zf - za) <= 1e-12 * np.linalg.norm(za)
    # the matrix-free operator is the dense Kronecker sum
    np.testing.assert_allclose(pre.matvec(r).reshape(-1), A @ r.reshape(-1),
                               atol=1e-12 * np.abs(A).max())
    # p = 2 with Dirichlet ends: S = S^reg, IFFD is exact (Sections 4, 7)
    if p == 2:
        np.testing.assert_allclose(P, A, atol=1e-12 * np.abs(A).max())
    # spectral equivalence (Proposition 1 with the constants of Theorem 1's
    # proof): a = 1 + 4 sqrt(3)/pi, c = 1/(a^2 + (1+a)^2), C = 2
    w = scipy.linalg.eigh(A, P, eigvals_only=True)
    a = 1 + 4 * np.sqrt(3) / np.pi
    bound = 2 * (a * a + (1 + a) ** 2)
    assert w.max() / w.min() <= bound


def test_kappa_flat_in_n_and_lanczos_agrees():
    # Lanczos estimate from PCG vs the dense generalized eigenvalues
    d, n, p = 2, 9, 3
    pre = iffd.Preconditioner(d, n, p, "iffd_a")
    A = brute.dense_system(pre.K, pre.M, d)
    P = brute.dense_preconditioner(pre.Kt, pre.M, d)
    w = scipy.linalg.eigh(A, P, eigvals_only=True)
    f = np.random.default_rng(0).uniform(-1, 1, (pre.m,) * d)
    out = krylov.pcg(pre.matvec, pre.apply, f, tol=1e-14, maxit=60)
    lmin, lmax, kap = krylov.kappa_estimate(out[4], out[5])
    # Ritz values lie inside the spectrum and approach its ends
    assert lmin >= w.min() * (1 - 1e-10) and lmax <= w.max() * (1 + 1e-10)
    assert kap <= w.max() / w.min() * (1 + 1e-10)
    assert kap >= 0.99 * w.max() / w.min()
    # robustness in h (Theorem 1): the estimate hardly moves with n
    kaps = []
    for n in (16, 32, 64):
        pre = iffd.Preconditioner(2, n, 3, "iffd_a")
        f = np.random.default_rng(1).uniform(-1, 1, (pre.m,) * 2)
        out = krylov.pcg(pre.matvec, pre.apply, f, tol=1e-13, maxit=40)
        kaps.append(krylov.kappa_estimate(out[4], out[5])[2])
    assert max(kaps) < 1.5 and max(kaps) / min(kaps) < 1.2
