"""Oracle pins for the variable-coefficient operator A_c (oracle/operator.py):
its 1-D stiffness against an independent B-spline library with adaptive
quadrature, the Kronecker assembly against explicit np.kron matrices, and
the Rayleigh-quotient bounds min c <= v^T A_c v / v^T A-hat v <= max c
(Section 3's bound on kappa(A-hat^{-1} A) with a diagonal coefficient)."""

import numpy as np
import pytest
from scipy import integrate, interpolate, linalg

from oracle import bspline
from oracle import operator as OP


def scipy_stiffness(n, p, a):
    """[K_c]_ij = int_0^1 (1 + a x) B_j' B_i' on S_{p,h,{0,1}}, from scipy's
    B-splines and adaptive quadrature element by element."""
    t = np.concatenate([np.zeros(p + 1), np.arange(1, n) / n, np.ones(p + 1)])
    nb = n + p
    dB = [interpolate.BSpline(t, np.eye(nb)[j], p).derivative() for j in range(nb)]
    K = np.zeros((nb, nb))
    for i in range(nb):
        for j in range(i, nb):
            if abs(i - j) > p:
                continue
            s = 0.0
            for e in range(n):
                s += integrate.quad(lambda x: (1 + a * x) * dB[i](x) * dB[j](x), e / n, (e + 1) / n,
                                    epsabs=1e-13, epsrel=1e-12)[0]
            K[i, j] = K[j, i] = s
    return K[1:-1, 1:-1]


@pytest.mark.parametrize("n,p,a", [(6, 2, 1.0), (7, 3, 0.5), (5, 4, 3.0), (9, 3, -0.6)])
def test_coefficient_stiffness_matches_independent_library(n, p, a):
    K = OP.Operator(2, n, p, a).K
    Ks = scipy_stiffness(n, p, a)
    assert np.max(np.abs(K - Ks)) <= 1e-12 * np.max(np.abs(Ks))


def test_zero_coefficient_is_the_laplacian():
    K0, M0 = bspline.assemble_dirichlet(10, 3)
    o = OP.Operator(3, 10, 3, 0.0)
    np.testing.assert_allclose(o.K, K0, rtol=0, atol=1e-14)
    np.testing.assert_array_equal(o.M, M0)


def test_operator_matches_explicit_kronecker_sum():
    rng = np.random.default_rng(3)
    for d, n, p, a in [(2, 7, 3, 1.0), (3, 5, 2, 2.5)]:
        o = OP.Operator(d, n, p, a)
        m = o.m
        K, M = o.K, o.M
        if d == 2:
            A = np.kron(M, K) + np.kron(K, M)
        else:
            A = np.kron(np.kron(M, M), K) + np.kron(np.kron(M, K), M) + np.kron(np.kron(K, M), M)
        X = rng.uniform(-1, 1, (m,) * d)
        np.testing.assert_allclose(o.matvec(X).ravel(), A @ X.ravel(), rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("a", [1.0, 4.0, -0.5])
def test_rayleigh_quotients_within_the_coefficient_range(a):
    """Generalized eigenvalues of (K_c, K) in 1-D and of (A_c, A-hat) in 2-D
    lie in [min c, max c] = [min(1, 1+a), max(1, 1+a)]; the extremes are
    approached as h -> 0."""
    lo, hi = min(1.0, 1.0 + a), max(1.0, 1.0 + a)
    n, p = 12, 3
    K0, M = bspline.assemble_dirichlet(n, p)
    Kc = OP.Operator(2, n, p, a).K
    ev = linalg.eigh(Kc, K0, eigvals_only=True)
    assert lo - 1e-12 <= ev.min() and ev.max() <= hi + 1e-12
    A0 = np.kron(M, K0) + np.kron(K0, M)
    Ac = np.kron(M, Kc) + np.kron(Kc, M)
    ev2 = linalg.eigh(Ac, A0, eigvals_only=True)
    assert lo - 1e-12 <= ev2.min() and ev2.max() <= hi + 1e-12
    # and the range is nearly filled (the coefficient's extremes are felt)
    assert ev2.max() - ev2.min() >= 0.8 * (hi - lo)


def test_planted_coefficient_error_is_caught():
    """A dropped factor in the quadrature weight (c applied twice) breaks the
    library comparison."""
    n, p, a = 6, 3, 1.0
    Kbad = bspline.assemble_dirichlet(n, p, lambda x: (1 + a * x) ** 2)[0]
    Ks = scipy_stiffness(n, p, a)
    assert np.max(np.abs(Kbad - Ks)) > 1e-3 * np.max(np.abs(Ks))
