"""Pins for oracle.krylov: CG against a direct solve, one iteration with an
exact preconditioner, and the printed iteration counts of Table 2."""

import json
import os

import numpy as np
import pytest

from oracle import iffd, krylov
import workloads

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table2_square.json")


def test_cg_matches_direct_solve():
    rng = np.random.default_rng(7)
    X = rng.standard_normal((40, 40))
    A = X @ X.T + 40 * np.eye(40)
    f = rng.standard_normal(40)
    u, it, conv, hist, _, _ = krylov.pcg(lambda v: A @ v, lambda v: v, f, tol=1e-13, maxit=200)
    assert conv
    np.testing.assert_allclose(u, np.linalg.solve(A, f), rtol=1e-10)
    # exact preconditioner: one step
    Ai = np.linalg.inv(A)
    u, it, conv, *_ = krylov.pcg(lambda v: A @ v, lambda v: Ai @ v, f, tol=1e-8)
    assert conv and it == 1


def test_zero_rhs():
    u, it, conv, *_ = krylov.pcg(lambda v: v, lambda v: v, np.zeros(5))
    assert conv and it == 0 and not u.any()


def test_fd_solves_in_one_iteration():
    pre = iffd.Preconditioner(2, 32, 4, "fd")
    f = workloads.uniform_rhs(2, 32, 4, 11)
    _, it, conv, *_ = krylov.pcg(pre.matvec, pre.apply, f)
    assert conv and it == 1


@pytest.mark.parametrize("col", range(6))
def test_table2_iterations(col):
    g = json.load(open(GOLDEN))
    n = g["n"][0]
    p = g["p"][col]
    printed = g["iterations"][0][col]
    pre = iffd.Preconditioner(2, n, p, "iffd_a")
    f = workloads.uniform_rhs(2, n, p, 1)
    u, it, conv, hist, _, _ = krylov.pcg(pre.matvec, pre.apply, f, tol=1e-8)
    assert conv
    if p == 2:
        assert it == printed == 1
    else:
        assert abs(it - printed) <= 1
    # the true residual agrees with the recursive one
    res = np.linalg.norm(f - pre.matvec(u)) / np.linalg.norm(f)
    assert res <= 1.5e-8
