"""GPU parity of the mapped-domain system matrix (Section 2's problem on
Omega = F([0,1]^3), Section 7's thick quarter of annulus) against the
oracle's assembled Galerkin matrix (oracle/geometry.py), and PCG with the
A-hat preconditioners on it (Section 3: the preconditioner is built from the
parameter-domain matrix; Table 4).

Tolerance: the operator is FP64 on both sides and differs only in the order
of the sums (sum factorization and a fixed-order gather here, dense local
matrices there): 1e-13 relative in the 2-norm and the max-norm.  PCG in FP64
takes the same number of iterations as the oracle's on the same right-hand
side; Table 4's counts are reproduced within +-1 (tests/golden)."""

import functools
import json
import os

import numpy as np
import pytest

import workloads
from oracle import general as G
from oracle import geometry as Gm
from oracle import krylov

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2512_20269_amd as I  # noqa: E402
from test_gpu_parity import dev, host, rel  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
DSET = {(1, 1): {0, 1}, (1, 0): {0}, (0, 1): {1}, (0, 0): set()}
ANNULUS = ("annulus", (1.0, 2.0, 1.0))
PLATE = ("plate", workloads.PLATE_PARAMS)
BOTTOM = ((0, 0), (0, 0), (1, 0))   # Dirichlet on the face xi_3 = 0 only


def specs_of(n, p, dl):
    return tuple((nk, pk, frozenset(DSET[tuple(dk)])) for nk, pk, dk in zip(n, p, dl))


@functools.lru_cache(maxsize=None)
def geo_oracle(specs, geometry):
    return Gm.GeometryOperator([(n, p, set(D)) for n, p, D in specs], geometry[0], geometry[1])


def make_plan(n, p, dl, geometry, method="fft", prec="f64", max_rhs=1):
    if dl is None:   # a uniform plan: Dirichlet everywhere, one n and p
        return I.Plan(3, n, p, method=method, precision=prec, max_rhs=max_rhs,
                      geometry=geometry)
    return I.Plan(3, list(n), list(p), method=method, precision=prec, max_rhs=max_rhs,
                  dirichlet=[tuple(x) for x in dl], geometry=geometry)


def plan_specs(n, p, dl):
    if dl is None:
        return specs_of((n,) * 3, (p,) * 3, ((1, 1),) * 3)
    return specs_of(n, p, dl)


# (n, p, ends or None for a uniform Dirichlet plan, geometry, method)
MATVEC_CASES = [
    (8, 2, None, ("bump", (0.05,)), "fft"),
    (8, 3, None, ("bump", (-0.08,)), "fft"),
    (12, 4, None, ("bump", (0.03,)), "dense"),
    ((8, 12, 16), (2, 3, 4), ((1, 0), (0, 1), (0, 0)), ("bump", (0.06,)), "fft"),
    ((8, 8, 8), (2, 2, 2), BOTTOM, ANNULUS, "fft"),
    ((8, 8, 8), (5, 5, 5), BOTTOM, ANNULUS, "fft"),
    ((12, 8, 16), (3, 4, 2), BOTTOM, ANNULUS, "fft"),
    ((16, 8, 8), (1, 3, 2), ((1, 1), (0, 0), (1, 0)), ("annulus", (0.5, 3.0, 2.0)), "fft"),
    # one degree in all directions from p = 1 to p = 8 (the line-wise element kernel)
    ((16, 8, 8), (1, 1, 1), BOTTOM, ANNULUS, "fft"),
    ((8, 8, 8), (4, 4, 4), ((1, 0), (0, 1), (0, 0)), ("bump", (-0.04,)), "fft"),
    ((8, 8, 8), (6, 6, 6), BOTTOM, ANNULUS, "fft"),
    ((8, 8, 8), (7, 7, 7), ((0, 0), (1, 1), (0, 1)), ("bump", (0.09,)), "fft"),
    # the plate with a hole (C^0 map across xi_1 = 1/2) on the smooth space
    ((8, 8, 8), (3, 3, 3), BOTTOM, PLATE, "fft"),
    ((12, 8, 16), (2, 4, 3), BOTTOM, PLATE, "dense"),
]


@pytest.mark.parametrize("n,p,dl,geometry,method", MATVEC_CASES)
def test_geometry_matvec_matches_oracle(n, p, dl, geometry, method):
    op = geo_oracle(plan_specs(n, p, dl), geometry)
    pl = make_plan(n, p, dl, geometry, method=method, max_rhs=2)
    assert pl.shape == op.shape
    X = np.stack([workloads.uniform_tensor(pl.shape, seed=s) for s in (3, 4)])
    y = host(pl.matvec(dev(X)))
    yo = op.matvec(X)
    e2, emax = rel(y, yo), float(np.abs(y - yo).max() / np.abs(yo).max())
    print(f"geometry {geometry[0]} n={n} p={p} ends={dl} {method}: rel2 {e2:.2e} max {emax:.2e}",
          flush=True)
    assert e2 <= 1e-13 and emax <= 1e-13


def greville(n, p):
    knots = np.concatenate([np.zeros(p + 1), np.arange(1, n) / n, np.ones(p + 1)])
    return np.array([knots[i + 1:i + p + 1].mean() for i in range(n + p)])


@pytest.mark.parametrize("p", [7, 8])
def test_geometry_high_degree_properties(p):
    """Where the oracle's dense assembly is out of reach (p = 8 needs n >= 12):
    the energy of u = x_3 = H xi_3 (in the space: it vanishes on the Dirichlet
    face xi_3 = 0) is the volume of the domain up to the quadrature error, and
    the operator is symmetric."""
    n = 12
    r_in, r_out, H = 1.0, 2.0, 1.5
    pl = make_plan((n,) * 3, (p,) * 3, BOTTOM, ("annulus", (r_in, r_out, H)), max_rhs=2)
    g3 = greville(n, p)[1:]   # kept B-splines of direction 3 (Dirichlet at 0)
    U = np.broadcast_to(H * g3[:, None, None], pl.shape).copy()
    e = float(np.vdot(U, host(pl.matvec(dev(U)))))
    vol = np.pi / 4 * (r_out ** 2 - r_in ** 2) * H
    X = np.stack([workloads.uniform_tensor(pl.shape, seed=s) for s in (11, 12)])
    Y = host(pl.matvec(dev(X)))
    asym = abs(np.vdot(X[0], Y[1]) - np.vdot(Y[0], X[1])) / (np.linalg.norm(X[0]) * np.linalg.norm(Y[1]))
    print(f"p={p}: energy {e:.15f} vs volume {vol:.15f}, asymmetry {asym:.1e}", flush=True)
    assert abs(e - vol) <= 1e-9 * vol
    assert asym <= 1e-14


def test_geometry_matvec_is_deterministic_and_batched():
    n, p, dl = (12, 8, 16), (3, 4, 2), BOTTOM
    pl = make_plan(n, p, dl, ANNULUS, max_rhs=3)
    X = np.stack([workloads.uniform_tensor(pl.shape, seed=s) for s in (5, 6, 7)])
    y3 = host(pl.matvec(dev(X)))
    y1 = host(pl.matvec(dev(X[1:2])))
    assert np.array_equal(y3[1:2], y1)
    assert np.array_equal(y3, host(pl.matvec(dev(X))))


# (n, p, ends, geometry, method, oracle preconditioner)
PCG_CASES = [
    (8, 3, None, ("bump", (0.07,)), "fft", "iffd_b"),
    (8, 3, None, ("bump", (0.07,)), "dense", "fd"),
    ((16, 16, 16), (2, 2, 2), BOTTOM, ANNULUS, "fft", "iffd_b"),
    ((16, 16, 16), (3, 3, 3), BOTTOM, ANNULUS, "fft", "iffd_b"),
]


@pytest.mark.parametrize("n,p,dl,geometry,method,kind", PCG_CASES)
def test_geometry_pcg_matches_oracle(n, p, dl, geometry, method, kind):
    specs = plan_specs(n, p, dl)
    op = geo_oracle(specs, geometry)
    pre = G.GeneralPreconditioner([(a, b, set(D)) for a, b, D in specs], kind)
    pl = make_plan(n, p, dl, geometry, method=method, prec="f64")
    f = workloads.uniform_tensor(pl.shape, seed=1)
    uo, it_o, conv_o, hist, *_ = krylov.pcg(op.matvec, pre.apply, f, tol=1e-8, maxit=200)
    u, st = pl.solve(dev(f), rtol=1e-8, maxit=200)
    s = st[0]
    u = host(u)
    print(f"PCG {geometry[0]} n={n} p={p} {method}: {s['iterations']} iterations "
          f"(oracle {it_o}), relres {s['relres']:.3e} (oracle {hist[-1]:.3e})", flush=True)
    assert conv_o and s["converged"]
    assert s["iterations"] == it_o
    assert abs(s["relres"] - hist[-1]) <= 1e-6 * hist[-1]
    assert rel(u, uo) <= 1e-9


@pytest.mark.parametrize("n", [16, 32, 64])
def test_table4_iffd_counts_on_gpu(n):
    """Table 4 (thick quarter of annulus, Dirichlet on the bottom face,
    natural elsewhere): IFFD PCG iterations with the FP32 apply within +-1
    of the printed counts for p = 2..5."""
    g = json.load(open(os.path.join(HERE, "golden", "table4_annulus.json")))
    printed = g["iffd"][g["n"].index(n)]
    for p, it_p in zip(g["p"], printed):
        pl = make_plan((n,) * 3, (p,) * 3, BOTTOM, ANNULUS, prec="f32")
        f = workloads.uniform_tensor(pl.shape, seed=1)
        _, st = pl.solve(dev(f), rtol=1e-8, maxit=200)
        s = st[0]
        print(f"Table 4 n={n} p={p}: IFFD {s['iterations']} (printed {it_p})", flush=True)
        assert s["converged"] and abs(s["iterations"] - it_p) <= 1
        del pl
        torch.cuda.empty_cache()


@pytest.mark.parametrize("p", [2, 3])
def test_annulus_fd_pcg_matches_oracle(p):
    """Dense FD (exact eigendecompositions) preconditioning the annulus
    operator: the oracle's FD PCG iterations, FP64."""
    n = (16, 16, 16)
    specs = plan_specs(n, (p,) * 3, BOTTOM)
    op = geo_oracle(specs, ANNULUS)
    pre = G.GeneralPreconditioner([(a, b, set(D)) for a, b, D in specs], "fd")
    pl = make_plan(n, (p,) * 3, BOTTOM, ANNULUS, method="dense", prec="f64")
    f = workloads.uniform_tensor(pl.shape, seed=1)
    _, it_o, conv_o, hist, *_ = krylov.pcg(op.matvec, pre.apply, f, tol=1e-8, maxit=200)
    _, st = pl.solve(dev(f), rtol=1e-8, maxit=200)
    print(f"annulus FD n={n} p={p}: {st[0]['iterations']} (oracle {it_o})", flush=True)
    assert conv_o and st[0]["converged"] and st[0]["iterations"] == it_o


@pytest.mark.parametrize("n", [16, 32, 64])
def test_table4_fd_counts_on_gpu(n):
    """Table 4's FD column (exact eigendecompositions, FP32 mode products on
    the matrix cores): within +-1 of the printed counts for p = 2..5."""
    g = json.load(open(os.path.join(HERE, "golden", "table4_annulus.json")))
    printed = g["fd"][g["n"].index(n)]
    for p, it_p in zip(g["p"], printed):
        pl = make_plan((n,) * 3, (p,) * 3, BOTTOM, ANNULUS, method="dense", prec="f32")
        f = workloads.uniform_tensor(pl.shape, seed=1)
        _, st = pl.solve(dev(f), rtol=1e-8, maxit=200)
        s = st[0]
        print(f"Table 4 n={n} p={p}: FD {s['iterations']} (printed {it_p})", flush=True)
        assert s["converged"] and abs(s["iterations"] - it_p) <= 1
        del pl
        torch.cuda.empty_cache()


# (n, p, ends, {direction: (k, mult)}, geometry): a repeated breakpoint
# (Remark rmk:reduced_regularity) under a map, through both element kernels
KNOT_CASES = [
    ((12, 8, 16), (2, 3, 2), BOTTOM, {1: (6, 2), 3: (8, 2)}, ANNULUS),
    ((12, 12, 12), (3, 3, 3), BOTTOM, {2: (6, 3)}, ANNULUS),
    ((12, 12, 12), (3, 3, 3), ((1, 0), (0, 1), (0, 0)), {1: (6, 2), 3: (6, 3)}, ("bump", (0.06,))),
    ((16, 12, 12), (4, 4, 4), BOTTOM, {1: (8, 4)}, ANNULUS),
    # the plate with the space C^0 across its corner plane, as its map
    ((12, 8, 16), (3, 2, 2), BOTTOM, {1: (6, 3)}, PLATE),
    ((16, 12, 12), (4, 4, 4), BOTTOM, {1: (8, 4)}, PLATE),
]


def knot_specs(n, p, dl, knots):
    return [(nk, pk, set(DSET[tuple(dk)]), knots.get(k + 1))
            for k, (nk, pk, dk) in enumerate(zip(n, p, dl))]


def knot_plan(n, p, dl, knots, geometry, method="fft", prec="f64", max_rhs=1):
    return I.Plan(3, list(n), list(p), method=method, precision=prec, max_rhs=max_rhs,
                  dirichlet=[tuple(x) for x in dl], geometry=geometry, knots=knots)


@pytest.mark.parametrize("n,p,dl,knots,geometry", KNOT_CASES)
def test_geometry_matvec_with_repeated_knot_matches_oracle(n, p, dl, knots, geometry):
    op = Gm.GeometryOperator(knot_specs(n, p, dl, knots), geometry[0], geometry[1])
    pl = knot_plan(n, p, dl, knots, geometry, max_rhs=2)
    assert pl.shape == op.shape
    X = np.stack([workloads.uniform_tensor(pl.shape, seed=s) for s in (8, 9)])
    y = host(pl.matvec(dev(X)))
    yo = op.matvec(X)
    e2, emax = rel(y, yo), float(np.abs(y - yo).max() / np.abs(yo).max())
    print(f"geometry {geometry[0]} n={n} p={p} knots={knots}: rel2 {e2:.2e} max {emax:.2e}",
          flush=True)
    assert e2 <= 1e-13 and emax <= 1e-13


@pytest.mark.parametrize("method,kind", [("fft", "iffd_b"), ("dense", "fd")])
def test_annulus_pcg_with_c0_plane_matches_oracle(method, kind):
    """The thick quarter of annulus with a C^0 plane at xi_1 = 1/2 (the
    breakpoint repeated p times): PCG with IFFD on the reduced space (the
    knot's extra outlier functions) or dense FD, against the oracle's PCG
    with the same preconditioner, FP64: the same iteration count."""
    from oracle import reduced as R
    n, p, knots = (16, 16, 16), (3, 3, 3), {1: (8, 3)}
    specs = knot_specs(n, p, BOTTOM, knots)
    op = Gm.GeometryOperator(specs, *ANNULUS)
    pre = R.ReducedPreconditioner(specs, kind)
    pl = knot_plan(n, p, BOTTOM, knots, ANNULUS, method=method)
    f = workloads.uniform_tensor(pl.shape, seed=1)
    uo, it_o, conv_o, hist, *_ = krylov.pcg(op.matvec, pre.apply, f, tol=1e-8, maxit=200)
    u, st = pl.solve(dev(f), rtol=1e-8, maxit=200)
    s = st[0]
    print(f"annulus C^0 plane {method}: {s['iterations']} iterations (oracle {it_o})", flush=True)
    assert conv_o and s["converged"]
    assert s["iterations"] == it_o
    assert rel(host(u), uo) <= 1e-9


@pytest.mark.parametrize("method,kind", [("fft", "iffd_b"), ("dense", "fd")])
def test_plate_c0_pcg_matches_oracle(method, kind):
    """The plate with a hole, its map only C^0 across xi_1 = 1/2 and the
    spline space C^0 there too (the breakpoint repeated p times, Remark
    rmk:reduced_regularity): PCG with IFFD on the reduced space or dense FD
    against the oracle's PCG, FP64: the same iteration count."""
    from oracle import reduced as R
    n, p, knots = (16, 16, 16), (3, 3, 3), {1: (8, 3)}
    specs = knot_specs(n, p, BOTTOM, knots)
    op = Gm.GeometryOperator(specs, *PLATE)
    pre = R.ReducedPreconditioner(specs, kind)
    pl = knot_plan(n, p, BOTTOM, knots, PLATE, method=method)
    f = workloads.uniform_tensor(pl.shape, seed=1)
    uo, it_o, conv_o, hist, *_ = krylov.pcg(op.matvec, pre.apply, f, tol=1e-8, maxit=200)
    u, st = pl.solve(dev(f), rtol=1e-8, maxit=200)
    s = st[0]
    print(f"plate C^0 {method}: {s['iterations']} iterations (oracle {it_o})", flush=True)
    assert conv_o and s["converged"]
    assert s["iterations"] == it_o
    assert rel(host(u), uo) <= 1e-9


def test_plate_c0_counts_robust_on_gpu():
    """The plate with a hole and a C^0 space across its corner plane (a
    stand-in for Table 5, whose plate comes from a geometry file that is not
    available): PCG iterations to 1e-8 with IFFD (FP32 apply) and dense FD
    for n = 32, 64, 128 and p = 2..5.  As in Table 5 the counts barely move
    with n (at most 3 apart for each p and method) and IFFD needs nearly the
    iterations of FD: Table 5 has IFFD within 7% of FD; this geometry is not
    the paper's, and IFFD is allowed 15% (observed up to 11%, at p = 2)."""
    counts = {}
    for n in (32, 64, 128):
        for p in (2, 3, 4, 5):
            for method in ("fft", "dense"):
                pl = knot_plan((n,) * 3, (p,) * 3, BOTTOM, {1: (n // 2, p)}, PLATE,
                               method=method, prec="f32")
                f = workloads.uniform_tensor(pl.shape, seed=1)
                _, st = pl.solve(dev(f), rtol=1e-8, maxit=300)
                assert st[0]["converged"], (n, p, method)
                counts[n, p, method] = st[0]["iterations"]
                del pl, f
                torch.cuda.empty_cache()
            print(f"plate C^0 n={n} p={p}: FD {counts[n, p, 'dense']} / IFFD {counts[n, p, 'fft']}",
                  flush=True)
    for p in (2, 3, 4, 5):
        for method in ("fft", "dense"):
            c = [counts[n, p, method] for n in (32, 64, 128)]
            assert max(c) - min(c) <= 3, (p, method, c)
        for n in (32, 64, 128):
            assert counts[n, p, "fft"] <= 1.15 * counts[n, p, "dense"], (n, p)


def test_geometry_state_rules():
    pl = make_plan(8, 2, None, ("bump", (0.05,)))
    rc = I.lib.iffd_plan_set_geometry(pl._h, I.GEOMETRY_NONE, None, 0)
    assert rc == I.E_STATE   # after setup


# ---- 2D mapped domains (the cross sections of the maps) ---------------------
# (n, p, ends, knots, geometry)
MATVEC2_CASES = [
    ((12, 16), (2, 3), ((1, 0), (0, 0)), {}, ("bump", (0.06,))),
    ((16, 16), (3, 3), ((0, 0), (1, 0)), {}, ("annulus", (1.0, 2.0))),
    ((16, 12), (4, 2), ((0, 0), (1, 0)), {1: (8, 4)}, ("plate", (1.0, 2.0))),
    ((8, 8), (1, 1), ((1, 1), (1, 1)), {}, ("plate", (1.0, 2.0))),
    ((24, 16), (5, 3), ((1, 1), (1, 1)), {1: (12, 5)}, ("plate", (1.0, 2.0))),
]


def plan2(n, p, dl, knots, geometry, method="fft", prec="f64", max_rhs=1):
    return I.Plan(2, list(n), list(p), method=method, precision=prec, max_rhs=max_rhs,
                  dirichlet=[tuple(x) for x in dl], geometry=geometry, knots=knots or None)


def specs2(n, p, dl, knots):
    return [(nk, pk, set(DSET[tuple(dk)]), knots.get(k + 1))
            for k, (nk, pk, dk) in enumerate(zip(n, p, dl))]


@pytest.mark.parametrize("n,p,dl,knots,geometry", MATVEC2_CASES)
def test_2d_geometry_matvec_matches_oracle(n, p, dl, knots, geometry):
    op = Gm.GeometryOperator(specs2(n, p, dl, knots), *geometry)
    pl = plan2(n, p, dl, knots, geometry, max_rhs=2)
    assert pl.shape == op.shape
    X = np.stack([workloads.uniform_tensor(pl.shape, seed=s) for s in (5, 6)])
    y = host(pl.matvec(dev(X)))
    yo = op.matvec(X)
    e2, emax = rel(y, yo), float(np.abs(y - yo).max() / np.abs(yo).max())
    print(f"2D geometry {geometry[0]} n={n} p={p} knots={knots}: rel2 {e2:.2e} max {emax:.2e}",
          flush=True)
    assert e2 <= 1e-13 and emax <= 1e-13


@pytest.mark.parametrize("method,kind", [("fft", "iffd_b"), ("dense", "fd")])
def test_2d_plate_c0_pcg_matches_oracle(method, kind):
    """The 2D plate with a hole (Dirichlet on the whole boundary) on the space
    C^0 across its corner line: PCG in FP64 takes the oracle's iterations."""
    from oracle import reduced as R
    n, p, dl, knots = (32, 32), (3, 3), ((1, 1), (1, 1)), {1: (16, 3)}
    specs = specs2(n, p, dl, knots)
    op = Gm.GeometryOperator(specs, "plate", workloads.PLATE_PARAMS[:2])
    pre = R.ReducedPreconditioner(specs, kind)
    pl = plan2(n, p, dl, knots, ("plate", workloads.PLATE_PARAMS[:2]), method=method)
    f = workloads.uniform_tensor(pl.shape, seed=1)
    uo, it_o, conv_o, hist, *_ = krylov.pcg(op.matvec, pre.apply, f, tol=1e-8, maxit=300)
    u, st = pl.solve(dev(f), rtol=1e-8, maxit=300)
    s = st[0]
    print(f"2D plate C^0 {method}: {s['iterations']} iterations (oracle {it_o})", flush=True)
    assert conv_o and s["converged"]
    assert s["iterations"] == it_o
    assert rel(host(u), uo) <= 1e-9


def test_2d_plate_c0_counts_robust_on_gpu():
    """Table 5's sizes in its own dimension (2D, n = 64, 128, 256, p = 2..5,
    the space C^0 across the plate's corner line, Dirichlet on the whole
    boundary): FD and IFFD (FP32 applies) iterations to 1e-8 at most 3 apart
    over n for each p and method, IFFD within 15% of FD (Table 5: within 7%;
    the plate here is not the paper's)."""
    counts = {}
    for n in (64, 128, 256):
        for p in (2, 3, 4, 5):
            for method in ("fft", "dense"):
                pl = plan2((n, n), (p, p), ((1, 1), (1, 1)), {1: (n // 2, p)},
                           ("plate", workloads.PLATE_PARAMS[:2]), method=method, prec="f32")
                f = workloads.uniform_tensor(pl.shape, seed=1)
                _, st = pl.solve(dev(f), rtol=1e-8, maxit=300)
                assert st[0]["converged"], (n, p, method)
                counts[n, p, method] = st[0]["iterations"]
                del pl, f
                torch.cuda.empty_cache()
            print(f"2D plate C^0 n={n} p={p}: FD {counts[n, p, 'dense']} / IFFD {counts[n, p, 'fft']}",
                  flush=True)
    for p in (2, 3, 4, 5):
        for method in ("fft", "dense"):
            c = [counts[n, p, method] for n in (64, 128, 256)]
            assert max(c) - min(c) <= 3, (p, method, c)
        for n in (64, 128, 256):
            assert counts[n, p, "fft"] <= 1.15 * counts[n, p, "dense"], (n, p)


@pytest.mark.parametrize("n,p,geometry,method", [
    (16, 3, ("bump", (0.05,)), "fft"),
    (16, 2, ("annulus", (1.0, 2.0)), "fft"),
    (24, 4, ("plate", (1.0, 2.0)), "dense"),
])
def test_2d_uniform_plan_geometry_matches_oracle(n, p, geometry, method):
    """2D mapped domains on a uniform plan (Dirichlet on every side, one n
    and p), operator and FP64 PCG iterations against the oracle."""
    specs = [(n, p, {0, 1})] * 2
    op = Gm.GeometryOperator(specs, *geometry)
    pl = I.Plan(2, n, p, method=method, precision="f64", geometry=geometry)
    assert pl.shape == op.shape
    X = workloads.uniform_tensor(pl.shape, seed=7)
    y, yo = host(pl.matvec(dev(X))), op.matvec(X)
    assert rel(y, yo) <= 1e-13
    pre = G.GeneralPreconditioner([(n, p, {0, 1})] * 2, "iffd_b" if method == "fft" else "fd")
    _, it_o, conv_o, *_ = krylov.pcg(op.matvec, pre.apply, X, tol=1e-8, maxit=300)
    _, st = pl.solve(dev(X), rtol=1e-8, maxit=300)
    print(f"2D uniform {geometry[0]} n={n} p={p} {method}: {st[0]['iterations']} (oracle {it_o})",
          flush=True)
    assert conv_o and st[0]["converged"] and st[0]["iterations"] == it_o


@pytest.mark.parametrize("geometry,d", [(ANNULUS, 3), (PLATE, 3), (("plate", (1.0, 2.0)), 2)])
def test_fd_kappa_within_section3_bound(geometry, d):
    """Section 3: with FD (the exact inverse of A-hat) the preconditioned
    operator's spectrum lies inside the extremes of G over the quadrature
    points, so the PCG's Lanczos estimate of kappa(A-hat^{-1} A) is at most
    max G / min G (eigenvalues of G at every Gauss point, from the oracle's
    map)."""
    n, p = 16, 2
    dl = BOTTOM if d == 3 else ((1, 1), (1, 1))
    specs = [(n, p, set(DSET[tuple(x)])) for x in dl]
    pl = I.Plan(d, [n] * d, [p] * d, method="dense", precision="f64",
                dirichlet=[tuple(x) for x in dl], geometry=geometry)
    f = workloads.uniform_tensor(pl.shape, seed=3)
    _, st = pl.solve(dev(f), rtol=1e-10, maxit=300)
    pts = [Gm.element_tables(nk, pk)[0].reshape(-1) for nk, pk, _ in specs]
    X = np.stack(np.meshgrid(*pts, indexing="ij"), axis=-1).reshape(-1, d)
    ev = np.linalg.eigvalsh(Gm.coefficient(geometry[0], geometry[1], X))
    bound = ev.max() / ev.min()
    print(f"{geometry[0]} {d}D: kappa_est {st[0]['kappa_est']:.3f}, Section 3 bound {bound:.3f}",
          flush=True)
    assert st[0]["converged"]
    assert 1.0 < st[0]["kappa_est"] <= bound * (1 + 1e-6)


def test_2d_geometry_matvec_is_deterministic_and_batched():
    """The 2D operator (one-point third direction, PM^2 items per workgroup):
    a batch member's result equals its single right-hand side result bit for
    bit, and repeated calls agree bit for bit."""
    n, p, dl, knots = (24, 16), (3, 2), ((1, 1), (0, 1)), {1: (12, 3)}
    pl = plan2(n, p, dl, knots, ("plate", (1.0, 2.0)), max_rhs=3)
    X = np.stack([workloads.uniform_tensor(pl.shape, seed=s) for s in (21, 22, 23)])
    y3 = host(pl.matvec(dev(X)))
    y1 = host(pl.matvec(dev(X[2:3])))
    assert np.array_equal(y3[2:3], y1)
    assert np.array_equal(y3, host(pl.matvec(dev(X))))
