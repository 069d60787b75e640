"""The Galerkin matrix of the Poisson problem on a mapped domain, the system
matrix A != A-hat that the paper preconditions with FD and IFFD built from
A-hat (Section 2, the problem on Omega = F([0,1]^3); Section 3, the bound on
kappa(A-hat^{-1} A); Section 7, the thick quarter of annulus).

Test infrastructure only (see the package docstring).

Pulled back to the parameter cube, the bilinear form is
    a(u, v) = int_[0,1]^3 grad v^T G grad u dxi,   G = |det J| J^{-1} J^{-T},
with J = dF/dxi (J[i][k] = d F_i / d xi_k), so
    A_ij = int grad B_i^T G grad B_j dxi
over the tensor-product B-splines B_i that the plan keeps (Dirichlet ends
drop their boundary B-spline, per direction).  The integrals use Gauss-
Legendre rules with p_k + 1 points per element and direction (Section 3's
rule; not exact here, G is not polynomial).

Synthetic maps (the paper's geometries come from GeoPDEs files that are not
available; these stand in for them):
  "bump"     F(xi) = xi + eps phi(xi) (1, 1, 1), phi = sin(pi xi_1) sin(pi
             xi_2) sin(pi xi_3): the unit cube itself (phi vanishes on its
             faces) with a non-separable interior parametrization, so A has no
             Kronecker structure; det J = 1 + eps (d1 phi + d2 phi + d3 phi).
  "annulus"  the thick quarter of annulus: F(xi) = (r c_1(t), r c_2(t), H xi_3)
             with r = r_in + (r_out - r_in) xi_1, t = xi_2 and c the quarter
             circle as a rational quadratic (control points (1,0), (1,1),
             (0,1), weights 1, 1/sqrt(2), 1), the exact NURBS form of the
             circle.
  "plate"    a quarter of a square plate [0, L]^2 with a hole of radius R at
             the corner, extruded to height H: F(xi) = ((1 - xi_2) R c(xi_1)
             + xi_2 o(xi_1), H xi_3), c the quarter circle as above and o the
             plate's two outer sides at constant speed, (L, 0) -> (L, L) ->
             (0, L), with the corner at xi_1 = 1/2.  F is only C^0 across the
             plane xi_1 = 1/2 (from the corner to the hole), the setting of
             Section 7's plate with hole (a C^0 line of the parametrization).
  "linear"   F(xi) = B xi for a fixed 3 x 3 matrix B (pins only).

In 2D (two specs, points with two coordinates) the maps are their cross
sections: the annulus and the plate without xi_3 (params (r_in, r_out) and
(R, L); a third value is ignored), the bump F = xi + eps sin(pi xi_1)
sin(pi xi_2) (1, 1), and "linear" with a 2 x 2 matrix.
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import bspline
from .general import kept


def jacobian(kind: str, params, X: np.ndarray) -> np.ndarray:
    """J at the points X (npts x d, d = 2 or 3): J[q, i, k] = d F_i / d xi_k."""
    X = np.asarray(X, dtype=np.float64)
    if X.shape[1] == 2:
        return _jacobian2(kind, params, X)
    npt = X.shape[0]
    J = np.zeros((npt, 3, 3))
    if kind == "bump":
        eps = float(params[0])
        s = np.sin(np.pi * X)
        c = np.cos(np.pi * X)
        grad = np.stack([np.pi * c[:, 0] * s[:, 1] * s[:, 2],
                         np.pi * s[:, 0] * c[:, 1] * s[:, 2],
                         np.pi * s[:, 0] * s[:, 1] * c[:, 2]], axis=1)
        for i in range(3):
            J[:, i, i] = 1.0
            J[:, i, :] += eps * grad
    elif kind == "annulus":
        r_in, r_out, H = (float(v) for v in params)
        t = X[:, 1]
        w = 1.0 / np.sqrt(2.0)
        b0, b1, b2 = (1 - t) ** 2, 2 * t * (1 - t), t ** 2
        db0, db1, db2 = -2 * (1 - t), 2 - 4 * t, 2 * t
        den = b0 + w * b1 + b2
        dden = db0 + w * db1 + db2
        n1 = b0 * 1.0 + w * b1 * 1.0 + b2 * 0.0
        n2 = b0 * 0.0 + w * b1 * 1.0 + b2 * 1.0
        dn1 = db0 + w * db1
        dn2 = w * db1 + db2
        c1, c2 = n1 / den, n2 / den
        dc1 = (dn1 * den - n1 * dden) / den ** 2
        dc2 = (dn2 * den - n2 * dden) / den ** 2
        r = r_in + (r_out - r_in) * X[:, 0]
        J[:, 0, 0] = (r_out - r_in) * c1
        J[:, 1, 0] = (r_out - r_in) * c2
        J[:, 0, 1] = r * dc1
        J[:, 1, 1] = r * dc2
        J[:, 2, 2] = H
    elif kind == "plate":
        R, Lp, H = (float(v) for v in params)
        t = X[:, 0]
        s = X[:, 1]
        w = 1.0 / np.sqrt(2.0)
        b0, b1, b2 = (1 - t) ** 2, 2 * t * (1 - t), t ** 2
        db0, db1, db2 = -2 * (1 - t), 2 - 4 * t, 2 * t
        den = b0 + w * b1 + b2
        dden = db0 + w * db1 + db2
        n1, n2 = b0 + w * b1, w * b1 + b2
        dn1, dn2 = db0 + w * db1, w * db1 + db2
        c1, c2 = n1 / den, n2 / den
        dc1 = (dn1 * den - n1 * dden) / den ** 2
        dc2 = (dn2 * den - n2 * dden) / den ** 2
        first = t < 0.5   # on the side x = L, else on the side y = L
        o1 = np.where(first, Lp, 2 * Lp * (1 - t))
        o2 = np.where(first, 2 * Lp * t, Lp)
        do1 = np.where(first, 0.0, -2 * Lp)
        do2 = np.where(first, 2 * Lp, 0.0)
        J[:, 0, 0] = (1 - s) * R * dc1 + s * do1
        J[:, 1, 0] = (1 - s) * R * dc2 + s * do2
        J[:, 0, 1] = o1 - R * c1
        J[:, 1, 1] = o2 - R * c2
        J[:, 2, 2] = H
    elif kind == "linear":
        Bm = np.asarray(params, dtype=np.float64).reshape(3, 3)
        J[:] = Bm
    else:
        raise ValueError(kind)
    return J


def _jacobian2(kind: str, params, X: np.ndarray) -> np.ndarray:
    """The 2D maps: the cross sections of the 3D ones."""
    npt = X.shape[0]
    if kind == "bump":
        eps = float(params[0])
        s, c = np.sin(np.pi * X), np.cos(np.pi * X)
        grad = np.stack([np.pi * c[:, 0] * s[:, 1], np.pi * s[:, 0] * c[:, 1]], axis=1)
        J = np.zeros((npt, 2, 2))
        for i in range(2):
            J[:, i, i] = 1.0
            J[:, i, :] += eps * grad
        return J
    if kind in ("annulus", "plate"):
        p3 = (float(params[0]), float(params[1]), 1.0)
        X3 = np.concatenate([X, np.zeros((npt, 1))], axis=1)
        return jacobian(kind, p3, X3)[:, :2, :2]
    if kind == "linear":
        return np.broadcast_to(np.asarray(params, dtype=np.float64).reshape(2, 2), (npt, 2, 2)).copy()
    raise ValueError(kind)


def coefficient(kind: str, params, X: np.ndarray) -> np.ndarray:
    """G = |det J| J^{-1} J^{-T} at the points X (npts x d x d)."""
    J = jacobian(kind, params, X)
    Ji = np.linalg.inv(J)
    det = np.abs(np.linalg.det(J))
    return det[:, None, None] * Ji @ np.transpose(Ji, (0, 2, 1))


def first_function(e: int, knot) -> int:
    """Full index of the first of the p+1 B-splines that are nonzero on element
    e: e, or e + mult - 1 past a breakpoint k/n repeated mult times."""
    if knot is None:
        return e
    k, mult = knot
    return e + (mult - 1 if e >= k else 0)


def element_tables(n: int, p: int, knot=None):
    """Per element e of one direction: the Gauss points (p+1), weights, and the
    values and derivatives of the p+1 B-splines nonzero there (full basis;
    knot = (k, mult) repeats the breakpoint k/n, Remark rmk:reduced_regularity)."""
    if knot is None:
        knots = bspline.open_knots(n, p)
    else:
        knots = np.sort(np.concatenate([bspline.open_knots(n, p),
                                        np.full(knot[1] - 1, knot[0] / n)]))
    gx, gw = np.polynomial.legendre.leggauss(p + 1)
    pts, wts, val, der = [], [], [], []
    for e in range(n):
        a, b = e / n, (e + 1) / n
        xq = 0.5 * (a + b) + 0.5 * (b - a) * gx
        f = first_function(e, knot)
        pts.append(xq)
        wts.append(0.5 * (b - a) * gw)
        val.append(bspline.basis(knots, p, xq)[:, f:f + p + 1])
        der.append(bspline.derivative(knots, p, xq, 1)[:, f:f + p + 1])
    return np.array(pts), np.array(wts), np.array(val), np.array(der)


def _spec(s):
    return (s[0], s[1], s[2], s[3] if len(s) > 3 else None)


def assemble2(specs, kind: str, params) -> sp.csr_matrix:
    """The 2D A over the kept tensor-product B-splines, index i1 + m1 i2,
    specs = [(n_k, p_k, D_k[, knot_k])] for k = 1, 2."""
    specs = [_spec(s) for s in specs]
    tabs = [element_tables(n, p, kt) for n, p, _, kt in specs]
    red, m = [], []
    for n, p, D, kt in specs:
        nb = n + p + (kt[1] - 1 if kt else 0)
        idx = np.arange(nb)
        if 0 in D:
            idx = idx[1:]
        if 1 in D:
            idx = idx[:-1]
        r = -np.ones(nb, dtype=np.int64)
        r[idx] = np.arange(len(idx))
        red.append(r)
        m.append(len(idx))
    rows, cols, vals = [], [], []
    (n1, p1, _, kt1), (n2, p2, _, kt2) = specs
    for e2 in range(n2):
        for e1 in range(n1):
            x1, w1, V1, D1 = (t[e1] for t in tabs[0])
            x2, w2, V2, D2 = (t[e2] for t in tabs[1])
            # points ordered (q2, q1)
            X = np.stack(np.meshgrid(x2, x1, indexing="ij")[::-1], axis=-1).reshape(-1, 2)
            W = np.outer(w2, w1).reshape(-1)
            G = coefficient(kind, params, X) * W[:, None, None]
            # gradients of the local functions (a2, a1) at the points (q2, q1)
            g1 = np.einsum("jb,ic->jibc", V2, D1)
            g2 = np.einsum("jb,ic->jibc", D2, V1)
            nq, nl = X.shape[0], (p1 + 1) * (p2 + 1)
            grad = np.stack([g1.reshape(nq, nl), g2.reshape(nq, nl)], axis=1)
            loc = grad.reshape(-1, nl).T @ np.einsum("qkl,qlj->qkj", G, grad).reshape(-1, nl)
            i2 = red[1][first_function(e2, kt2) + np.arange(p2 + 1)]
            i1 = red[0][first_function(e1, kt1) + np.arange(p1 + 1)]
            I2, I1 = np.meshgrid(i2, i1, indexing="ij")
            okf = ((I2 >= 0) & (I1 >= 0)).reshape(-1)
            li = np.nonzero(okf)[0]
            gi = (I1 + m[0] * I2).reshape(-1)[li]
            rows.append(np.repeat(gi, len(gi)))
            cols.append(np.tile(gi, len(gi)))
            vals.append(loc[np.ix_(li, li)].reshape(-1))
    N = m[0] * m[1]
    return sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(N, N)).tocsr()


def assemble(specs, kind: str, params) -> sp.csr_matrix:
    """A over the kept tensor-product B-splines, index i1 + m1 i2 + m1 m2 i3
    (direction 1 fastest), specs = [(n_k, p_k, D_k[, knot_k])] for k = 1, 2, 3
    (knot_k = (k, mult) or None); two specs give the 2D matrix."""
    if len(specs) == 2:
        return assemble2(specs, kind, params)
    assert len(specs) == 3
    specs = [_spec(s) for s in specs]
    tabs = [element_tables(n, p, kt) for n, p, _, kt in specs]
    nfull = [n + p + (kt[1] - 1 if kt else 0) for n, p, _, kt in specs]
    keep = []
    for (n, p, D, kt), nb in zip(specs, nfull):
        idx = np.arange(nb)
        if 0 in D:
            idx = idx[1:]
        if 1 in D:
            idx = idx[:-1]
        keep.append(idx)
    red = []
    for k in range(3):
        r = -np.ones(nfull[k], dtype=np.int64)
        r[keep[k]] = np.arange(len(keep[k]))
        red.append(r)
    m = [len(kk) for kk in keep]
    rows, cols, vals = [], [], []
    (n1, p1, _, kt1), (n2, p2, _, kt2), (n3, p3, _, kt3) = specs
    for e3 in range(n3):
        for e2 in range(n2):
            for e1 in range(n1):
                e = (e1, e2, e3)
                x = [tabs[k][0][e[k]] for k in range(3)]
                w = [tabs[k][1][e[k]] for k in range(3)]
                V = [tabs[k][2][e[k]] for k in range(3)]   # q_k x (p_k+1)
                Dv = [tabs[k][3][e[k]] for k in range(3)]
                # quadrature points, ordered (q3, q2, q1)
                X = np.stack(np.meshgrid(x[0], x[1], x[2], indexing="ij"), axis=-1)  # q1,q2,q3
                X = np.transpose(X, (2, 1, 0, 3)).reshape(-1, 3)
                W = np.einsum("c,b,a->cba", w[2], w[1], w[0]).reshape(-1)
                G = coefficient(kind, params, X) * W[:, None, None]
                # gradients of the local functions (a3, a2, a1) at the points (q3, q2, q1)
                g1 = np.einsum("ka,jb,ic->kjiabc", V[2], V[1], Dv[0])
                g2 = np.einsum("ka,jb,ic->kjiabc", V[2], Dv[1], V[0])
                g3 = np.einsum("ka,jb,ic->kjiabc", Dv[2], V[1], V[0])
                nq = X.shape[0]
                nl = (p1 + 1) * (p2 + 1) * (p3 + 1)
                grad = np.stack([g1.reshape(nq, nl), g2.reshape(nq, nl), g3.reshape(nq, nl)],
                                axis=1)   # nq x 3 x nl
                # loc_ij = sum_q sum_k,l grad[q,k,i] G[q,k,l] grad[q,l,j]
                Gg = np.einsum("qkl,qlj->qkj", G, grad)
                loc = grad.reshape(-1, nl).T @ Gg.reshape(-1, nl)
                # local -> reduced global indices
                i3 = red[2][first_function(e3, kt3) + np.arange(p3 + 1)]
                i2 = red[1][first_function(e2, kt2) + np.arange(p2 + 1)]
                i1 = red[0][first_function(e1, kt1) + np.arange(p1 + 1)]
                I3, I2, I1 = np.meshgrid(i3, i2, i1, indexing="ij")
                ok = (I3 >= 0) & (I2 >= 0) & (I1 >= 0)
                gidx = (I1 + m[0] * I2 + m[0] * m[1] * I3).reshape(-1)
                okf = ok.reshape(-1)
                li = np.nonzero(okf)[0]
                gi = gidx[li]
                rows.append(np.repeat(gi, len(gi)))
                cols.append(np.tile(gi, len(gi)))
                vals.append(loc[np.ix_(li, li)].reshape(-1))
    N = m[0] * m[1] * m[2]
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(N, N)).tocsr()
    return A


class GeometryOperator:
    """y = A x for a tensor of shape (m_3, m_2, m_1)."""

    def __init__(self, specs, kind: str, params):
        self.specs = [(int(s[0]), int(s[1]), frozenset(s[2]),
                       None if len(s) < 4 or s[3] is None else tuple(s[3])) for s in specs]
        self.kind, self.params = kind, tuple(float(v) for v in params)
        self.A = assemble(self.specs, kind, self.params)
        self.shape = tuple(len(kept(n, p, D)) + (kt[1] - 1 if kt else 0)
                           for n, p, D, kt in reversed(self.specs))

    def matvec(self, X: np.ndarray) -> np.ndarray:
        X = np.asarray(X, dtype=np.float64)
        lead = X.shape[:-len(self.shape)]
        Xf = X.reshape(-1, int(np.prod(self.shape)))
        Y = (self.A @ Xf.T).T
        return Y.reshape(lead + self.shape)
