"""Pins for oracle.bspline against closed forms and invariants that do not
come from the oracle's own formulas."""

from math import comb, factorial
from fractions import Fraction

import numpy as np
import pytest

from oracle import bspline


def truncated_power_cardinal(p, x):
    """Centered cardinal B-spline of degree p by the classical truncated
    power formula (Curry-Schoenberg):
    (1/p!) sum_k (-1)^k C(p+1,k) (x + (p+1)/2 - k)_+^p."""
    # evaluated at -|x| (the function is even): near the left end of the
    # support only a few terms are active, so the sum cancels least there
    x = -np.abs(np.asarray(x, dtype=np.float64))
    s = np.zeros_like(x)
    for k in range(p + 2):
        t = np.maximum(x + (p + 1) / 2 - k, 0.0)
        s += (-1) ** k * comb(p + 1, k) * (t ** p if p > 0 else (t > 0).astype(float))
    s[np.abs(x) >= (p + 1) / 2] = 0.0       # compact support
    return s / factorial(p)


@pytest.mark.parametrize("p", range(1, 10))
def test_cardinal_recurrence_matches_truncated_power(p):
    x = np.linspace(-(p + 2) / 2, (p + 2) / 2, 997)
    # avoid the break points for the degree-0/1 discontinuities
    x = x + 1e-7
    # the truncated power sum cancels catastrophically in the tails
    np.testing.assert_allclose(bspline.cardinal(p, x), truncated_power_cardinal(p, x),
                               atol=1e-10)


def test_cardinal_printed_values():
    # integer samples, Eulerian numbers / p!
    assert bspline.cardinal(3, np.array([-1.0, 0.0, 1.0])) == pytest.approx([1 / 6, 2 / 3, 1 / 6])
    assert bspline.cardinal(2, np.array([-1.0, 0.0, 1.0])) == pytest.approx([1 / 8, 3 / 4, 1 / 8])
    assert bspline.cardinal(4, 0.0) == pytest.approx(115 / 192)
    assert bspline.cardinal(4, 1.0) == pytest.approx(19 / 96)
    assert bspline.cardinal(4, 2.0) == pytest.approx(1 / 384)
    assert bspline.cardinal(5, 0.0) == pytest.approx(11 / 20)
    assert bspline.cardinal(5, 1.0) == pytest.approx(13 / 60)
    assert bspline.cardinal(7, 0.0) == pytest.approx(151 / 315)
    for p in range(1, 12):
        k = np.arange(-p, p + 1)
        assert bspline.cardinal(p, k.astype(float)).sum() == pytest.approx(1.0, abs=1e-14)


@pytest.mark.parametrize("p", range(1, 9))
def test_cox_de_boor_partition_of_unity_and_support(p):
    n = 11
    knots = bspline.open_knots(n, p)
    assert len(knots) == n + 2 * p + 1
    x = np.concatenate([np.linspace(0, 1, 301), [1.0]])
    B = bspline.basis(knots, p, x)
    assert B.shape == (len(x), n + p)
    np.testing.assert_allclose(B.sum(axis=1), 1.0, atol=1e-13)
    assert (B >= -1e-15).all()
    # interpolation at the ends: only the first/last function is nonzero
    assert B[0, 0] == pytest.approx(1.0) and B[-1, -1] == pytest.approx(1.0)
    # support of B_i is [xi_i, xi_{i+p+1}]
    for i in range(n + p):
        out = (x < knots[i] - 1e-12) | (x > knots[i + p + 1] + 1e-12)
        assert np.abs(B[out, i]).max(initial=0) == 0.0


@pytest.mark.parametrize("p", range(1, 9))
def test_derivatives_match_finite_differences(p):
    n = 7
    knots = bspline.open_knots(n, p)
    # points away from the knots (where the spline is smooth)
    x = (np.arange(n) + 0.37) / n
    eps = 1e-5
    for k in range(1, min(p, 3) + 1):
        lo = bspline.derivative(knots, p, x - eps, k - 1)
        hi = bspline.derivative(knots, p, x + eps, k - 1)
        fd = (hi - lo) / (2 * eps)
        ex = bspline.derivative(knots, p, x, k)
        scale = max(1.0, np.abs(ex).max())
        np.testing.assert_allclose(ex, fd, atol=1e-5 * scale * n ** k)


@pytest.mark.parametrize("p", range(1, 9))
def test_interior_bsplines_are_shifted_cardinals(p):
    n = 3 * p + 4
    h = 1.0 / n
    knots = bspline.open_knots(n, p)
    x = np.linspace(0, 1, 503)
    B = bspline.basis(knots, p, x)
    # B_l with l >= p and l + p + 1 <= n + p has support [(l-p)h, (l+1)h],
    # centre (l - p + (p+1)/2) h
    for l in range(p, n):
        c = l - p + (p + 1) / 2
        np.testing.assert_allclose(B[:, l], truncated_power_cardinal(p, x / h - c), atol=1e-11)


@pytest.mark.parametrize("p", range(1, 9))
def test_mass_stiffness_invariants_and_symbols(p):
    n = 4 * p + 6
    h = 1.0 / n
    K, M = bspline.assemble_full(n, p)
    knots = bspline.open_knots(n, p)
    np.testing.assert_allclose(K, K.T, atol=1e-13 * n)
    np.testing.assert_allclose(M, M.T, atol=1e-16 * n)
    # integral of B_i = (xi_{i+p+1} - xi_i) / (p+1)
    np.testing.assert_allclose(M.sum(axis=1), (knots[p + 1:] - knots[:n + p]) / (p + 1),
                               atol=1e-15)
    # constants are in the kernel of the full stiffness matrix
    np.testing.assert_allclose(K.sum(axis=1), 0.0, atol=1e-11 * n)
    # interior rows: the mass symbol h * B_{2p+1}(k) and the stiffness
    # symbol -(1/h) second difference of B_{2p-1}
    i = n // 2 + p // 2
    k = np.arange(-p, p + 1)
    m_row = h * truncated_power_cardinal(2 * p + 1, k.astype(float))
    b = lambda t: truncated_power_cardinal(2 * p - 1, t.astype(float))
    k_row = -(b(k + 1) - 2 * b(k) + b(k - 1)) / h
    np.testing.assert_allclose(M[i, i - p:i + p + 1], m_row, atol=1e-15)
    np.testing.assert_allclose(K[i, i - p:i + p + 1], k_row, rtol=1e-11, atol=1e-10)
    # Dirichlet-reduced matrices are SPD
    Kd, Md = bspline.assemble_dirichlet(n, p)
    assert Kd.shape == (n + p - 2, n + p - 2)
    assert np.linalg.eigvalsh(Md).min() > 0 and np.linalg.eigvalsh(Kd).min() > 0


def test_printed_low_degree_rows():
    n = 10
    h = 1.0 / n
    K, M = bspline.assemble_full(n, 1)
    np.testing.assert_allclose(M[4, 3:6], h / 6 * np.array([1, 4, 1]), atol=1e-16)
    np.testing.assert_allclose(K[4, 3:6], np.array([-1, 2, -1]) / h, atol=1e-12)
    K, M = bspline.assemble_full(n, 2)
    np.testing.assert_allclose(M[5, 3:8], h / 120 * np.array([1, 26, 66, 26, 1]), atol=1e-16)
    np.testing.assert_allclose(K[5, 3:8], np.array([-1, -2, 6, -2, -1]) / (6 * h), atol=1e-12)
