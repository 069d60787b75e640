"""Pins for oracle.reduced, IFFD with reduced regularity at an interior knot
(Remark rmk:reduced_regularity, eq:reg_space2).

  * dimensions: n_reg as for the maximally smooth space, n_out larger by one
    per extra copy of the knot (the remark's count), the constraint rows of
    route A (end conditions plus the derivative jumps at the knot) as many as
    n_out;
  * the special basis written on the B-splines of the reduced space meets
    every constraint (its functions are C^{p-1} at the knot);
  * the jump rows vanish on the maximally smooth space embedded by knot
    insertion (they measure exactly the lost smoothness);
  * route A (definition) = route B (structure);
  * mult = 1 is oracle.general's route B;
  * kappa(P^{-1} K) stays bounded and flat in n with a C^0 knot (the
    stable splitting of Theorem 2 carries over).
"""

import numpy as np
import pytest
import scipy.linalg as sla

from oracle import bspline
from oracle import general as G
from oracle import reduced as R

CASES = [frozenset(s) for s in ({0, 1}, {0}, {1}, set())]


def ids(D):
    return "D" + "".join(map(str, sorted(D)))


@pytest.mark.parametrize("D", CASES, ids=ids)
@pytest.mark.parametrize("p,mult", [(2, 2), (3, 2), (3, 3), (4, 4), (5, 3), (6, 6)])
def test_dimensions_constraints_and_routes(p, mult, D):
    n = 4 * p + 8
    k = n // 2
    m, n_reg, n_out = R.dims(n, p, D, mult)
    m0, n_reg0, n_out0 = G.dims(n, p, D)
    assert m == m0 + mult - 1 and n_reg == n_reg0 and n_out == n_out0 + mult - 1
    E = R.constraint_rows(n, p, D, k, mult)
    assert E.shape == (n_out, m)
    fb = R.factors_route_b(n, p, D, k, mult)
    V = fb["V_reg"]
    assert V.shape == (m, n_reg) and np.linalg.matrix_rank(V) == n_reg
    assert np.abs(E @ V).max() < 1e-12
    lam_a, Qa, K, M = R.factors_route_a(n, p, D, k, mult)
    r = np.random.default_rng(p + mult).standard_normal(m)
    za = Qa @ ((Qa.T @ r) / (lam_a + 1.0))
    zb = fb["Qt"] @ ((fb["Qt"].T @ r) / (fb["lam_t"] + 1.0))
    assert np.abs(za - zb).max() <= 1e-10 * np.abs(zb).max()


@pytest.mark.parametrize("p", [2, 3, 5])
def test_jump_rows_vanish_on_the_smooth_space(p):
    """A function of the maximally smooth space, written on the B-splines of
    the space with the repeated knot (by collocation), has no derivative
    jumps there; a B-spline of the reduced space that is only C^{p-mult} at
    the knot has one."""
    n, k, mult = 12, 6, p
    kn = R.knots(n, p, k, mult)
    xs = (np.arange(400) + 0.5) / 400
    Bsm = bspline.basis(bspline.open_knots(n, p), p, xs)
    Bred = bspline.basis(kn, p, xs)
    C, *_ = np.linalg.lstsq(Bred, Bsm, rcond=None)   # smooth B-splines in the reduced basis
    assert np.abs(Bred @ C - Bsm).max() < 1e-12
    E = R.constraint_rows(n, p, set(), k, mult)
    jumps = E[-(mult - 1):]
    assert np.abs(jumps @ C).max() < 1e-10
    assert np.abs(jumps).max() > 0.1


@pytest.mark.parametrize("D", CASES, ids=ids)
@pytest.mark.parametrize("p", [2, 3, 4])
def test_single_knot_is_the_smooth_route(p, D):
    n = 16
    fb = R.factors_route_b(n, p, D, n // 2, 1)
    gb = G.factors_route_b(n, p, D)
    r = np.random.default_rng(p).standard_normal(fb["Qt"].shape[0])
    z1 = fb["Qt"] @ ((fb["Qt"].T @ r) / (fb["lam_t"] + 1.0))
    z2 = gb["Qt"] @ ((gb["Qt"].T @ r) / (gb["lam_t"] + 1.0))
    assert np.abs(z1 - z2).max() <= 1e-11 * np.abs(z2).max()


@pytest.mark.parametrize("p", [2, 3, 4, 5])
def test_condition_number_flat_with_a_c0_knot(p):
    kap = []
    for n in (16, 32, 64):
        fb = R.factors_route_b(n, p, {0, 1}, n // 2, p)
        Pinv = fb["Qt"] @ np.diag(1 / fb["lam_t"]) @ fb["Qt"].T
        ev = np.sort(np.real(sla.eigvals(Pinv @ fb["K"])))
        kap.append(ev[-1] / ev[0])
    assert max(kap) < 1.5 and abs(kap[-1] - kap[-2]) < 0.05, kap
