"""Pins for oracle.geometry, the Galerkin matrix on a mapped domain (Section
2's problem on Omega = F([0,1]^3); Section 3's bound on kappa(A-hat^{-1} A);
Section 7's thick quarter of annulus, Table 4).

  * eps = 0 (the identity map) gives A-hat, the Kronecker sum of the exact
    one-dimensional stiffness and mass matrices;
  * F(xi) = B xi with a non-symmetric B: the energy of u = a . F(xi) (exactly
    representable with natural ends) is |a|^2 |det B|, the integral of
    |grad_x u|^2 over B([0,1]^3); a transposed or inverted G fails it;
  * the annulus: the energies of u = x_3 = H xi_3 and of the radial u = xi_1
    are vol(Omega) and vol(Omega) / (r_out - r_in)^2 (quadrature error only);
  * the Jacobians against central differences of the maps, written here from
    their definitions (the rational quadratic as a weighted sum of the three
    control points, which is a quarter of the unit circle);
  * Section 3's bound: every generalized eigenvalue of (A, A-hat) lies in
    [min lambda_min(G), max lambda_max(G)] over the quadrature points (the
    rule integrates |grad u|^2 exactly, so the bound holds without slack);
  * Table 4's iteration counts at n = 16, p = 2, for FD and IFFD.
"""

import json
import os

import numpy as np
import pytest
import scipy.linalg as sla

import workloads
from oracle import geometry as Gm
from oracle import general as G
from oracle import krylov

HERE = os.path.dirname(os.path.abspath(__file__))
ANNULUS = (1.0, 2.0, 1.0)


def bump_map(eps, X):
    phi = np.prod(np.sin(np.pi * X), axis=1)
    return X + eps * phi[:, None]


def circle_arc(t):
    """The rational quadratic with control points (1,0), (1,1), (0,1) and
    weights 1, 1/sqrt(2), 1, as the weighted sum of its control points."""
    P = np.array([[1.0, 0.0], [1.0, 1.0], [0.0, 1.0]])
    w = np.array([1.0, 1.0 / np.sqrt(2.0), 1.0])
    B = np.stack([(1 - t) ** 2, 2 * t * (1 - t), t ** 2], axis=1) * w
    return (B @ P) / B.sum(axis=1)[:, None]


def annulus_map(par, X):
    r_in, r_out, H = par
    r = r_in + (r_out - r_in) * X[:, 0]
    c = circle_arc(X[:, 1])
    return np.stack([r * c[:, 0], r * c[:, 1], H * X[:, 2]], axis=1)


PLATE = (1.0, 2.0, 1.0)   # hole radius R, plate side L, height H


def plate_map(par, X):
    """(1 - xi_2) R c(xi_1) + xi_2 o(xi_1), o walking the two outer sides
    (L, 0) -> (L, L) -> (0, L) at constant speed; x_3 = H xi_3."""
    R, Lp, H = par
    t, s = X[:, 0], X[:, 1]
    c = circle_arc(t)
    o = np.where((t < 0.5)[:, None], np.stack([np.full_like(t, Lp), 2 * Lp * t], axis=1),
                 np.stack([2 * Lp * (1 - t), np.full_like(t, Lp)], axis=1))
    xy = (1 - s)[:, None] * R * c + s[:, None] * o
    return np.stack([xy[:, 0], xy[:, 1], H * X[:, 2]], axis=1)


def fd_jacobian(F, X, h=1e-6):
    J = np.zeros((X.shape[0], 3, 3))
    for k in range(3):
        E = np.zeros(3)
        E[k] = h
        J[:, :, k] = (F(X + E) - F(X - E)) / (2 * h)
    return J


def test_maps_jacobians_against_differences():
    X = np.random.default_rng(0).uniform(0.05, 0.95, (40, 3))
    Jb = Gm.jacobian("bump", [0.07], X)
    assert np.abs(Jb - fd_jacobian(lambda Y: bump_map(0.07, Y), X)).max() < 1e-8
    Ja = Gm.jacobian("annulus", ANNULUS, X)
    assert np.abs(Ja - fd_jacobian(lambda Y: annulus_map(ANNULUS, Y), X)).max() < 1e-8
    t = np.linspace(0, 1, 101)
    c = circle_arc(t)
    assert np.abs(np.hypot(c[:, 0], c[:, 1]) - 1).max() < 1e-15   # a quarter of the unit circle
    assert np.allclose(c[0], [1, 0]) and np.allclose(c[-1], [0, 1])
    # the plate: away from its C^0 plane xi_1 = 1/2 (differences must not
    # straddle the corner)
    Xp = X[np.abs(X[:, 0] - 0.5) > 0.01]
    Jp = Gm.jacobian("plate", PLATE, Xp)
    assert np.abs(Jp - fd_jacobian(lambda Y: plate_map(PLATE, Y), Xp)).max() < 1e-8
    # its faces: the hole xi_2 = 0 on the circle of radius R, xi_2 = 1 on the
    # sides x = L or y = L with the corner at xi_1 = 1/2
    e = np.linspace(0, 1, 41)
    hole = plate_map(PLATE, np.stack([e, 0 * e, 0 * e], axis=1))
    side = plate_map(PLATE, np.stack([e, 0 * e + 1, 0 * e], axis=1))
    assert np.abs(np.hypot(hole[:, 0], hole[:, 1]) - PLATE[0]).max() < 1e-14
    assert np.abs(np.maximum(side[:, 0], side[:, 1]) - PLATE[1]).max() < 1e-14
    assert np.allclose(side[20, :2], [PLATE[1], PLATE[1]])
    # the derivative along xi_1 jumps across the plane: only C^0 there
    Jl = Gm.jacobian("plate", PLATE, np.array([[0.5 - 1e-12, 0.7, 0.3]]))
    Jr = Gm.jacobian("plate", PLATE, np.array([[0.5 + 1e-12, 0.7, 0.3]]))
    assert np.abs(Jl[0, :2, 0] - Jr[0, :2, 0]).max() > 1.0
    assert np.abs(Jl[0, :, 1:] - Jr[0, :, 1:]).max() < 1e-9
    # no fold: det J keeps one sign over the cube (negative: xi_1 runs along
    # the arc, xi_2 outwards)
    Xg = np.random.default_rng(1).uniform(0, 1, (400, 3))
    assert np.linalg.det(Gm.jacobian("plate", PLATE, Xg)).max() < -0.1
    # G is |det J| (J^T J)^{-1}: symmetric positive definite
    Gq = Gm.coefficient("annulus", ANNULUS, X)
    assert np.abs(Gq - np.transpose(Gq, (0, 2, 1))).max() < 1e-14
    assert np.linalg.eigvalsh(Gq).min() > 0


@pytest.mark.parametrize("p", [1, 2, 3])
def test_identity_map_gives_A_hat(p):
    n = 5
    specs = [(n, p, {0, 1}), (n + 1, p, {0}), (n, p, set())]
    A = Gm.GeometryOperator(specs, "bump", [0.0])
    Ahat = G.GeneralPreconditioner(specs, "fd")
    X = np.random.default_rng(p).standard_normal(A.shape)
    ref = Ahat.matvec(X)
    assert A.shape == Ahat.shape
    assert np.abs(A.matvec(X) - ref).max() <= 1e-13 * np.abs(ref).max()


@pytest.mark.parametrize("p", [1, 2, 3])
def test_linear_map_energy(p):
    B = np.array([[1.3, 0.4, -0.2], [0.1, 0.9, 0.3], [-0.5, 0.2, 1.7]])
    n = 4
    specs = [(n, p, set())] * 3
    A = Gm.GeometryOperator(specs, "linear", B.reshape(-1))
    # Greville abscissae reproduce linear functions: u(xi) = sum_i g_i B_i(xi) = xi
    knots = np.concatenate([np.zeros(p + 1), np.arange(1, n) / n, np.ones(p + 1)])
    g = np.array([knots[i + 1:i + p + 1].mean() for i in range(n + p)])
    G3, G2, G1 = np.meshgrid(g, g, g, indexing="ij")   # (i3, i2, i1)
    a = np.array([0.7, -1.1, 0.4])
    c = a @ B   # u = a . (B xi) = (a B) . xi
    U = c[0] * G1 + c[1] * G2 + c[2] * G3
    energy = float(np.vdot(U, A.matvec(U)))
    exact = float(a @ a) * abs(np.linalg.det(B))
    assert abs(energy - exact) <= 1e-12 * exact
    # constants carry no energy (natural ends)
    assert np.abs(A.matvec(np.ones(A.shape))).max() < 1e-12


def test_annulus_energies():
    r_in, r_out, H = ANNULUS
    vol = np.pi / 4 * (r_out ** 2 - r_in ** 2) * H
    n, p = 6, 2
    specs = [(n, p, set())] * 3
    A = Gm.GeometryOperator(specs, "annulus", ANNULUS)
    knots = np.concatenate([np.zeros(p + 1), np.arange(1, n) / n, np.ones(p + 1)])
    g = np.array([knots[i + 1:i + p + 1].mean() for i in range(n + p)])
    G3, G2, G1 = np.meshgrid(g, g, g, indexing="ij")
    e3 = float(np.vdot(H * G3, A.matvec(H * G3)))   # u = x_3: |grad u| = 1
    e1 = float(np.vdot(G1, A.matvec(G1)))           # u = (r - r_in) / (r_out - r_in)
    assert abs(e3 - vol) < 1e-6 * vol
    assert abs(e1 - vol / (r_out - r_in) ** 2) < 1e-6 * vol


def test_plate_energy():
    """The energy of u = x_3 = H xi_3 over the plate with a hole is its
    volume (L^2 - pi R^2 / 4) H, up to the quadrature error of the rational
    map; n_1 even puts the corner plane on a breakpoint."""
    R, Lp, H = PLATE
    vol = (Lp ** 2 - np.pi * R ** 2 / 4) * H
    n, p = 6, 2
    A = Gm.GeometryOperator([(n, p, set())] * 3, "plate", PLATE)
    knots = np.concatenate([np.zeros(p + 1), np.arange(1, n) / n, np.ones(p + 1)])
    g = np.array([knots[i + 1:i + p + 1].mean() for i in range(n + p)])
    G3 = np.broadcast_to(g[:, None, None], A.shape)
    e3 = float(np.vdot(H * G3, A.matvec(H * G3)))
    assert abs(e3 - vol) < 1e-5 * vol


@pytest.mark.parametrize("kind,par", [("bump", [0.08]), ("annulus", ANNULUS), ("plate", PLATE)])
def test_section3_bound(kind, par):
    n, p = 4, 2
    specs = [(n, p, {0, 1}), (n, p, {0, 1}), (n, p, {0})]
    A = Gm.GeometryOperator(specs, kind, par).A.toarray()
    Ahat = G.GeneralPreconditioner(specs, "fd")
    N = A.shape[0]
    Ah = np.stack([Ahat.matvec(e.reshape(Ahat.shape)).reshape(-1) for e in np.eye(N)], axis=1)
    assert np.abs(A - A.T).max() < 1e-13 * np.abs(A).max()
    lam = sla.eigh(A, Ah, eigvals_only=True)
    # the extremes of G over the quadrature points of every element
    pts = []
    for (nk, pk, _) in specs:
        x, _, _, _ = Gm.element_tables(nk, pk)
        pts.append(x.reshape(-1))
    X = np.stack(np.meshgrid(*pts, indexing="ij"), axis=-1).reshape(-1, 3)
    ev = np.linalg.eigvalsh(Gm.coefficient(kind, par, X))
    lo, hi = ev.min(), ev.max()
    assert lam.min() >= lo * (1 - 1e-10) and lam.max() <= hi * (1 + 1e-10)
    assert lam.max() / lam.min() > 1.0 + 1e-3   # A is not A-hat


def test_table4_annulus_n16_p2():
    gold = json.load(open(os.path.join(HERE, "golden", "table4_annulus.json")))
    n, p = 16, 2
    specs = [(n, p, set()), (n, p, set()), (n, p, {0})]   # Dirichlet on the bottom face xi_3 = 0
    A = Gm.GeometryOperator(specs, "annulus", ANNULUS)
    f = workloads.uniform_tensor(A.shape, seed=1)
    its = {}
    for kind in ("fd", "iffd_b"):
        pre = G.GeneralPreconditioner(specs, kind)
        _, it, conv, *_ = krylov.pcg(A.matvec, pre.apply, f, tol=1e-8, maxit=200)
        assert conv
        its[kind] = it
    i, j = gold["n"].index(n), gold["p"].index(p)
    assert abs(its["fd"] - gold["fd"][i][j]) <= 1, its
    assert abs(its["iffd_b"] - gold["iffd"][i][j]) <= 1, its


def _restriction(n, p, D, knot):
    """E with B^smooth_j = sum_i E_ij B^knot_i on the kept functions of one
    direction: the smooth spline space is a subspace of the space with the
    repeated breakpoint, so a least-squares fit at 7 points per element is
    exact."""
    from oracle import bspline, reduced as R
    xs = (np.arange(7 * n) + 0.5) / (7 * n)
    Bs = bspline.basis(bspline.open_knots(n, p), p, xs)[:, R.kept(n + p, D)]
    Bk = bspline.basis(R.knots(n, p, *knot), p, xs)[:, R.kept(n + p + knot[1] - 1, D)]
    E, *_ = np.linalg.lstsq(Bk, Bs, rcond=None)
    assert np.abs(Bk @ E - Bs).max() < 1e-12
    return E


@pytest.mark.parametrize("p,mult", [(2, 2), (3, 2), (3, 3)])
def test_repeated_knot_identity_map_gives_reduced_A_hat(p, mult):
    """With a breakpoint of multiplicity mult (Remark rmk:reduced_regularity)
    the identity map gives the Kronecker sum of the reduced space's exact
    one-dimensional K and M (assembled there over the whole basis, not per
    element): a wrong first function past the breakpoint fails it."""
    from oracle import reduced as R
    n = 8
    specs = [(n, p, {0, 1}, (4, mult)), (n, 2, {0}, None), (n + 1, p, set(), (3, mult))]
    A = Gm.GeometryOperator(specs, "bump", [0.0])
    X = np.random.default_rng(mult).standard_normal(A.shape)
    (K1, M1), (K2, M2), (K3, M3) = [R.assemble(nk, pk, D, *kt) if kt else _smooth_km(nk, pk, D)
                                    for nk, pk, D, kt in specs]
    Ahat = (np.kron(M3, np.kron(M2, K1)) + np.kron(M3, np.kron(K2, M1))
            + np.kron(K3, np.kron(M2, M1)))
    ref = (Ahat @ X.reshape(-1)).reshape(A.shape)
    assert A.shape == (M3.shape[0], M2.shape[0], M1.shape[0])
    assert np.abs(A.matvec(X) - ref).max() <= 1e-13 * np.abs(ref).max()


def _smooth_km(n, p, D):
    """K and M of the maximally smooth space by Gauss-Legendre over the whole
    basis (exact for the polynomial integrands)."""
    from oracle import bspline, reduced as R
    kn = bspline.open_knots(n, p)
    gx, gw = np.polynomial.legendre.leggauss(p + 1)
    K = np.zeros((n + p, n + p))
    M = np.zeros((n + p, n + p))
    for e in range(n):
        xq = (e + 0.5 + 0.5 * gx) / n
        wq = 0.5 * gw / n
        B = bspline.basis(kn, p, xq)
        dB = bspline.derivative(kn, p, xq, 1)
        M += (B * wq[:, None]).T @ B
        K += (dB * wq[:, None]).T @ dB
    kk = R.kept(n + p, D)
    return K[np.ix_(kk, kk)], M[np.ix_(kk, kk)]


@pytest.mark.parametrize("kind,par", [("bump", (0.05,)), ("annulus", ANNULUS), ("plate", PLATE)])
def test_repeated_knot_contains_smooth_operator(kind, par):
    """The maximally smooth space is a subspace of the space with a repeated
    breakpoint, and A is the same bilinear form on both: E^T A_knot E =
    A_smooth for any map, E the (Kronecker) inclusion of the coefficients."""
    n, p = 6, 3
    D = [{0, 1}, {0}, {0}]
    knots = [(3, 3), None, (2, 2)]
    Ak = Gm.GeometryOperator([(n, p, D[k], knots[k]) for k in range(3)], kind, par)
    As = Gm.GeometryOperator([(n, p, D[k]) for k in range(3)], kind, par)
    Es = []
    for k in range(3):
        if knots[k] is None:
            Es.append(np.eye(n + p - len(D[k])))
        else:
            Es.append(_restriction(n, p, D[k], knots[k]))
    E = np.kron(Es[2], np.kron(Es[1], Es[0]))
    lhs = E.T @ (Ak.A @ E)
    ref = As.A.toarray()
    assert np.abs(lhs - ref).max() <= 1e-12 * np.abs(ref).max()
    # and the knot space is strictly larger: A_knot is SPD on it
    w = np.linalg.eigvalsh(Ak.A.toarray())
    assert w.min() > 0


# ---- 2D: the cross sections of the maps ------------------------------------

@pytest.mark.parametrize("p", [1, 2, 3])
def test_2d_identity_map_gives_A_hat(p):
    specs = [(6, p, {0, 1}), (7, p, {0})]
    A = Gm.GeometryOperator(specs, "bump", [0.0])
    Ahat = G.GeneralPreconditioner(specs, "fd")
    X = np.random.default_rng(p).standard_normal(A.shape)
    ref = Ahat.matvec(X)
    assert A.shape == Ahat.shape
    assert np.abs(A.matvec(X) - ref).max() <= 1e-13 * np.abs(ref).max()


@pytest.mark.parametrize("p", [1, 2, 3])
def test_2d_linear_map_energy(p):
    """u = a . (B xi) over B([0,1]^2): energy |a|^2 |det B| (a transposed or
    inverted G, or points in the wrong order, fail it)."""
    B = np.array([[1.3, 0.4], [-0.3, 0.9]])
    n = 4
    A = Gm.GeometryOperator([(n, p, set()), (n + 1, p, set())], "linear", B.reshape(-1))
    g1 = greville(n, p)
    g2 = greville(n + 1, p)
    G2, G1 = np.meshgrid(g2, g1, indexing="ij")
    a = np.array([0.7, -1.1])
    c = a @ B
    U = c[0] * G1 + c[1] * G2
    e = float(np.vdot(U, A.matvec(U)))
    exact = float(a @ a) * abs(np.linalg.det(B))
    assert abs(e - exact) <= 1e-12 * exact
    assert np.abs(A.matvec(np.ones(A.shape))).max() < 1e-12


def greville(n, p):
    knots = np.concatenate([np.zeros(p + 1), np.arange(1, n) / n, np.ones(p + 1)])
    return np.array([knots[i + 1:i + p + 1].mean() for i in range(n + p)])


def test_2d_maps():
    """The 2D maps' Jacobians against differences of their cross sections,
    the annulus' radial energy (area / (r_out - r_in)^2), one sign of det J
    on the plate, and its C^0 line xi_1 = 1/2."""
    X = np.random.default_rng(2).uniform(0.05, 0.95, (40, 2))
    X3 = np.concatenate([X, np.zeros((40, 1))], axis=1)
    Ja = Gm.jacobian("annulus", ANNULUS[:2], X)
    Fa = lambda Y: annulus_map(ANNULUS, np.concatenate([Y, np.zeros((len(Y), 1))], axis=1))[:, :2]
    assert np.abs(Ja - fd_jacobian2(Fa, X)).max() < 1e-8
    Xp = X[np.abs(X[:, 0] - 0.5) > 0.01]
    Fp = lambda Y: plate_map(PLATE, np.concatenate([Y, np.zeros((len(Y), 1))], axis=1))[:, :2]
    assert np.abs(Gm.jacobian("plate", PLATE[:2], Xp) - fd_jacobian2(Fp, Xp)).max() < 1e-8
    Jb = Gm.jacobian("bump", [0.07], X)
    Fb = lambda Y: Y + 0.07 * (np.sin(np.pi * Y[:, 0]) * np.sin(np.pi * Y[:, 1]))[:, None]
    assert np.abs(Jb - fd_jacobian2(Fb, X)).max() < 1e-8
    assert np.linalg.det(Gm.jacobian("plate", PLATE[:2], X)).max() < -0.1
    # the annulus' radial coordinate u = xi_1: |grad u| = 1 / (r_out - r_in)
    r_in, r_out, _ = ANNULUS
    n, p = 6, 2
    A = Gm.GeometryOperator([(n, p, set())] * 2, "annulus", ANNULUS[:2])
    g = greville(n, p)
    U = np.broadcast_to(g[None, :], A.shape)
    area = np.pi / 4 * (r_out ** 2 - r_in ** 2)
    assert abs(float(np.vdot(U, A.matvec(U))) - area / (r_out - r_in) ** 2) < 1e-6 * area
    del X3


def fd_jacobian2(F, X, h=1e-6):
    J = np.zeros((X.shape[0], 2, 2))
    for k in range(2):
        E = np.zeros(2)
        E[k] = h
        J[:, :, k] = (F(X + E) - F(X - E)) / (2 * h)
    return J


@pytest.mark.parametrize("kind,par", [("bump", [0.08]), ("annulus", ANNULUS[:2]), ("plate", PLATE[:2])])
def test_2d_section3_bound_and_c0_inclusion(kind, par):
    n, p = 6, 2
    specs = [(n, p, {0, 1}), (n, p, {0})]
    A = Gm.GeometryOperator(specs, kind, par).A.toarray()
    Ahat = G.GeneralPreconditioner(specs, "fd")
    N = A.shape[0]
    Ah = np.stack([Ahat.matvec(e.reshape(Ahat.shape)).reshape(-1) for e in np.eye(N)], axis=1)
    assert np.abs(A - A.T).max() < 1e-13 * np.abs(A).max()
    lam = sla.eigh(A, Ah, eigvals_only=True)
    pts = [Gm.element_tables(nk, pk)[0].reshape(-1) for nk, pk, _ in specs]
    Xq = np.stack(np.meshgrid(*pts, indexing="ij"), axis=-1).reshape(-1, 2)
    ev = np.linalg.eigvalsh(Gm.coefficient(kind, par, Xq))
    assert lam.min() >= ev.min() * (1 - 1e-10) and lam.max() <= ev.max() * (1 + 1e-10)
    # the smooth space inside the space with a C^0 line xi_1 = 1/2
    kn = (3, p)
    Ak = Gm.GeometryOperator([(n, p, {0, 1}, kn), (n, p, {0}, None)], kind, par)
    E = np.kron(np.eye(n + p - 1), _restriction(n, p, {0, 1}, kn))
    assert np.abs(E.T @ (Ak.A @ E) - A).max() <= 1e-12 * np.abs(A).max()


@pytest.mark.parametrize("d", [2, 3])
def test_annulus_energy_of_xi1_squared(d):
    """u = xi_1^2 (in the space for p >= 2) on the annulus, where G varies
    with xi_1 and xi_2: its energy against int (2 xi_1)^2 G_00 dxi by a fine
    tensor Gauss rule.  Unlike the constant-gradient energies this pairs each
    element's gradients with G at the right points (swapped point coordinates
    fail it)."""
    from oracle import bspline
    n, p = 5, 2
    par = ANNULUS[:2] if d == 2 else ANNULUS
    A = Gm.GeometryOperator([(n, p, set())] * d, "annulus", par)
    xs = np.linspace(0, 1, 61)
    B = bspline.basis(bspline.open_knots(n, p), p, xs)
    c1 = np.linalg.lstsq(B, xs ** 2, rcond=None)[0]
    assert np.abs(B @ c1 - xs ** 2).max() < 1e-13
    U = c1
    for _ in range(d - 1):
        U = np.multiply.outer(np.ones(n + p), U)   # constant along xi_2 (, xi_3)
    e = float(np.vdot(U, A.matvec(U)))
    gx, gw = np.polynomial.legendre.leggauss(40)
    t, w = 0.5 * (gx + 1), 0.5 * gw
    T1, T2 = np.meshgrid(t, t, indexing="ij")
    X = np.stack([T1.reshape(-1), T2.reshape(-1)] + ([np.zeros(T1.size)] if d == 3 else []), axis=1)
    G00 = Gm.coefficient("annulus", par, X)[:, 0, 0]
    exact = float(np.sum(np.outer(w, w).reshape(-1) * (2 * X[:, 0]) ** 2 * G00))
    assert abs(e - exact) < 1e-6 * exact
