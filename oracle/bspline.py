"""Univariate splines on a uniform grid: knots, B-spline values and
derivatives, 1-D mass and stiffness matrices, symmetric cardinal B-splines.

Test infrastructure only (see the package docstring).

Sources
    Section 2, definition of S_{p,h}, the p-open knot vector and the Cox-de
    Boor recursion (zero-denominator terms dropped).
    Section 3, the 1-D matrices [K]_{ij} = int B_j' B_i', [M]_{ij} = int B_j B_i.
    Lemma 4, recurrence (eq:cardinal) for the symmetric cardinal B-spline.
"""

from __future__ import annotations

import numpy as np


def open_knots(n: int, p: int) -> np.ndarray:
    """p-open uniform knot vector xi_0..xi_{n+2p} on [0,1] with h = 1/n
    (Section 2): p+1 zeros, the n-1 interior breakpoints k/n, p+1 ones."""
    interior = np.arange(1, n, dtype=np.float64) / n
    return np.concatenate([np.zeros(p + 1), interior, np.ones(p + 1)])


def _degree0(knots: np.ndarray, x: np.ndarray, left: bool = False) -> np.ndarray:
    """Indicator functions of the half-open knot spans [xi_i, xi_{i+1}).

    At the right end x = xi_last the half-open rule gives nothing; the value
    there is taken as the left limit, i.e. the last non-empty span counts.
    left=True takes the spans (xi_i, xi_{i+1}] instead: values are then the
    limits from the left at the knots (a derivative jump at an interior knot
    is the difference of the two)."""
    nspan = len(knots) - 1
    B = np.zeros((len(x), nspan))
    for i in range(nspan):
        a, b = knots[i], knots[i + 1]
        if b > a:
            B[:, i] = ((x > a) & (x <= b)) if left else ((x >= a) & (x < b))
    if not left:
        last = max(i for i in range(nspan) if knots[i + 1] > knots[i])
        B[x == knots[-1], last] = 1.0
    return B


def basis(knots: np.ndarray, p: int, x, left: bool = False) -> np.ndarray:
    """Values of all degree-p B-splines at the points x, shape (len(x), nb),
    nb = len(knots) - p - 1, by the Cox-de Boor recursion of Section 2
    (left=True: limits from the left at knots)."""
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    B = _degree0(knots, x, left)
    for q in range(1, p + 1):
        nb = len(knots) - q - 1
        Bn = np.zeros((len(x), nb))
        for i in range(nb):
            d1 = knots[i + q] - knots[i]
            d2 = knots[i + q + 1] - knots[i + 1]
            if d1 > 0:
                Bn[:, i] += (x - knots[i]) / d1 * B[:, i]
            if d2 > 0:
                Bn[:, i] += (knots[i + q + 1] - x) / d2 * B[:, i + 1]
        B = Bn
    return B


def derivative(knots: np.ndarray, p: int, x, k: int, left: bool = False) -> np.ndarray:
    """k-th derivative of all degree-p B-splines at x (shape (len(x), nb)).

    Uses the standard derivative formula of the recursion:
    D B_{q,i} = q/(xi_{i+q}-xi_i) B_{q-1,i} - q/(xi_{i+q+1}-xi_{i+1}) B_{q-1,i+1},
    applied k times, with vanishing denominators dropped as in Section 2."""
    if k == 0:
        return basis(knots, p, x, left)
    if k > p:
        x = np.atleast_1d(x)
        return np.zeros((len(x), len(knots) - p - 1))
    lower = derivative(knots, p - 1, x, k - 1, left)
    nb = len(knots) - p - 1
    out = np.zeros((lower.shape[0], nb))
    for i in range(nb):
        d1 = knots[i + p] - knots[i]
        d2 = knots[i + p + 1] - knots[i + 1]
        if d1 > 0:
            out[:, i] += p / d1 * lower[:, i]
        if d2 > 0:
            out[:, i] -= p / d2 * lower[:, i + 1]
    return out


def assemble_full(n: int, p: int, coef=None):
    """Mass and stiffness matrices of the full space S_{p,h} (size n+p),
    by Gauss-Legendre quadrature with p+1 points per element, which is exact
    for the degree-2p integrands (Section 3, eq:system_matrix's factors).
    coef: optional stiffness coefficient c(x), [K]_{ij} = int c B_j' B_i'
    (still exact for c of degree <= 3: the integrand has degree 2p - 2 + 3)."""
    knots = open_knots(n, p)
    nb = n + p
    gx, gw = np.polynomial.legendre.leggauss(p + 1)
    M = np.zeros((nb, nb))
    K = np.zeros((nb, nb))
    for e in range(n):
        a, b = e / n, (e + 1) / n
        xq = 0.5 * (a + b) + 0.5 * (b - a) * gx
        wq = 0.5 * (b - a) * gw
        B = basis(knots, p, xq)
        dB = derivative(knots, p, xq, 1)
        M += (B * wq[:, None]).T @ B
        wk = wq if coef is None else wq * coef(xq)
        K += (dB * wk[:, None]).T @ dB
    return K, M


def assemble_dirichlet(n: int, p: int, coef=None):
    """K and M on S_{p,h,{0,1}}: the two B-splines that do not vanish at the
    ends are removed (Section 2), leaving m = n+p-2 functions B_1..B_{n+p-2}."""
    K, M = assemble_full(n, p, coef)
    return K[1:-1, 1:-1].copy(), M[1:-1, 1:-1].copy()


def cardinal(p: int, x) -> np.ndarray:
    """Symmetric cardinal B-spline of degree p, by the recurrence of Lemma 4
    (eq:cardinal): B_0 = indicator of [-1/2, 1/2), and
    B_p(x) = (p+1+2x)/(2p) B_{p-1}(x+1/2) + (p+1-2x)/(2p) B_{p-1}(x-1/2)."""
    x = np.asarray(x, dtype=np.float64)
    if p == 0:
        return ((x >= -0.5) & (x < 0.5)).astype(np.float64)
    return ((p + 1 + 2 * x) / (2 * p) * cardinal(p - 1, x + 0.5)
            + (p + 1 - 2 * x) / (2 * p) * cardinal(p - 1, x - 0.5))
