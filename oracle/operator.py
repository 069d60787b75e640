"""A system matrix A != A-hat for PCG with the constant-coefficient
preconditioners: a variable-coefficient operator.

Test infrastructure only (see the package docstring).

The preconditioners of Section 3 (FD) and Section 4 onwards (IFFD) are built
from A-hat, the Galerkin matrix of the Laplacian on the parameter domain,
and are applied to the matrix A of the coefficient-weighted bilinear form of
Section 1 (the pulled-back form, whose coefficient is a matrix function of
x); Section 3 bounds kappa(A-hat^{-1} A) by the extreme eigenvalues of that
coefficient.  Reading used here (no geometry data): a synthetic diagonal
coefficient D(x) = diag(c(x_1), .., c(x_d)) with c(x) = 1 + a x, a > -1, so
that

    A_c = sum_k M x .. x K_c (slot k) x .. x M,   [K_c]_ij = int_0^1 c B_j' B_i',

stays a sum of Kronecker products (the same sum factorization applies) while
A_c != A-hat for a != 0, and

    min c <= v^T A_c v / v^T A-hat v <= max c,   kappa(A-hat^{-1} A_c) <= 1 + |a| / min(1, 1 + a).

Parity of PCG on A_c with the paper's preconditioners is unpinned by the
paper (its variable-coefficient tables need geometry data); A_c itself is
pinned by an independent B-spline library and the bounds above.
"""

from __future__ import annotations

import numpy as np

from . import bspline
from .iffd import kron_matvec


def coefficient(a: float):
    """c(x) = 1 + a x."""
    return lambda x: 1.0 + a * np.asarray(x, dtype=np.float64)


class Operator:
    """y = A_c x on [0,1]^d, Dirichlet on every face, all directions with the
    same (n, p) and the same coefficient c(x_k) = 1 + a x_k in direction k."""

    def __init__(self, d: int, n: int, p: int, a: float):
        if not a > -1.0:
            raise ValueError("the coefficient 1 + a x must stay positive on [0,1]")
        self.d, self.n, self.p, self.a = d, n, p, a
        self.K, self.M = bspline.assemble_dirichlet(n, p, coefficient(a))
        self.m = self.K.shape[0]

    def matvec(self, X: np.ndarray) -> np.ndarray:
        d = self.d
        return kron_matvec(X, [self.K] * d, [self.M] * d, d)
