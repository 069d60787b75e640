"""GPU parity of the small 2-D route of the IFFD apply (eq:preconditioner
with Qt = [V_reg U Dt^{-1}, V_out Q_out] of Sections 4 and 6 held densely,
two launches of LDS products) against the oracle's route B, and against the
line passes on the same input.  FP32 tolerance 1e-5 as for the passes
(relative 2-norm, max-norm and boundary-slab RMS, test_gpu_parity.check).
The cases cover the uniform Dirichlet plans from the smallest n up to the
largest eligible m (98, at n = 96 and p = 4), p = 1 (no outliers), the end
conditions of Table 1 with anisotropic (n_k, p_k), repeated interior knots
(eq:reg_space2) along either direction, ragged slices (m not a multiple of
the 8-row slices) and batches, whose members get the same bits as alone."""
import functools

import numpy as np
import pytest

import workloads
from oracle import general as G
from oracle import krylov
from oracle import reduced as R

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
import paper_2512_20269_amd as I  # noqa: E402
from test_gpu_parity import check, dev, host, oracle, rel  # noqa: E402

TOL = 1e-5
DSET = {(1, 1): {0, 1}, (1, 0): {0}, (0, 1): {1}, (0, 0): set()}


def routes_agree(pl, r, zo, d, p, what):
    """The dense route matches the oracle, and the passes on the same input."""
    assert pl.route() == "dense2d", what
    z = host(pl.apply(dev(r)))
    check(z, zo, TOL, d, p, f"dense2d {what}")
    pl.set_route("passes")
    try:
        zp = host(pl.apply(dev(r)))
    finally:
        pl.set_route("auto")
    check(zp, zo, TOL, d, p, f"passes {what}")
    assert rel(z, zp) <= TOL
    return z


UNIFORM = [(8, 1), (8, 3), (12, 2), (16, 3), (16, 4), (24, 1), (32, 2), (48, 3), (64, 3),
           (64, 4), (96, 3), (96, 4)]


@pytest.mark.parametrize("n,p", UNIFORM)
def test_dense2d_uniform_matches_oracle(n, p):
    pl = I.Plan(2, n, p, precision="f32", max_rhs=3)
    R3 = workloads.batched_uniform_rhs(2, n, p, [n + p, n + p + 1, n + p + 2])
    print(f"dense2d uniform n={n} p={p}", flush=True)
    zo = np.stack([oracle(2, n, p).apply(R3[k]) for k in range(3)])
    routes_agree(pl, R3, zo, 2, p, f"n={n} p={p}")


GENERAL = [
    ((16, 24), (3, 3), ((1, 0), (1, 1))),
    ((16, 24), (4, 2), ((0, 0), (1, 1))),
    ((24, 16), (2, 4), ((0, 1), (1, 0))),
    ((12, 16), (1, 4), ((0, 0), (1, 0))),
    ((48, 32), (2, 3), ((1, 1), (0, 0))),
    ((96, 64), (3, 4), ((0, 1), (1, 0))),
    ((96, 96), (4, 4), ((0, 0), (0, 1))),   # m = 100 and 99
]


@pytest.mark.parametrize("n,p,dl", GENERAL)
def test_dense2d_general_matches_oracle(n, p, dl):
    pre = G.GeneralPreconditioner([(nk, pk, DSET[dk]) for nk, pk, dk in zip(n, p, dl)], "iffd_b")
    pl = I.Plan(2, list(n), list(p), precision="f32", dirichlet=list(dl))
    assert pl.shape == pre.shape
    r = workloads.uniform_tensor(pre.shape, seed=sum(n) + 10 * sum(p) + 1)
    print(f"dense2d general n={n} p={p} {dl}", flush=True)
    routes_agree(pl, r, pre.apply(r), 2, max(p), f"n={n} p={p} {dl}")


KNOTS = [
    ((32, 24), (3, 3), ((1, 1), (1, 1)), {1: (16, 3)}),   # C^0 along direction 1
    ((32, 48), (4, 2), ((1, 0), (0, 1)), {2: (24, 2)}),   # along direction 2, mult 2
    ((48, 48), (3, 4), ((0, 0), (1, 1)), {1: (12, 2), 2: (36, 4)}),
]


@pytest.mark.parametrize("n,p,dl,knots", KNOTS)
def test_dense2d_repeated_knot_matches_oracle(n, p, dl, knots):
    specs = [(nk, pk, DSET[dk], knots.get(k + 1)) for k, (nk, pk, dk) in enumerate(zip(n, p, dl))]
    pre = R.ReducedPreconditioner(specs, "iffd_b")
    pl = I.Plan(2, list(n), list(p), precision="f32", dirichlet=list(dl), knots=knots)
    assert pl.shape == pre.shape
    r = workloads.uniform_tensor(pre.shape, seed=sum(n) + 7)
    print(f"dense2d knot n={n} p={p} {dl} {knots}", flush=True)
    routes_agree(pl, r, pre.apply(r), 2, max(p), f"n={n} p={p} {dl} {knots}")


def test_dense2d_batch_members_equal_single_bitwise():
    n, p = 64, 3
    pl1 = I.Plan(2, n, p, precision="f32")
    plb = I.Plan(2, n, p, precision="f32", max_rhs=30)
    Rb = workloads.batched_uniform_rhs(2, n, p, list(range(50, 80)))
    assert pl1.route() == plb.route(30) == "dense2d"
    zb = host(plb.apply(dev(Rb)))
    for k in (0, 17, 29):
        assert np.array_equal(host(pl1.apply(dev(Rb[k]))), zb[k]), k
    assert np.array_equal(host(plb.apply(dev(Rb[3:9]))), zb[3:9])


def test_dense2d_noalloc_and_pcg():
    """The allocation-free apply takes the same route (same bits); a general
    plan's PCG, whose preconditioner applies run unfused and so take the dense
    route, matches the oracle's PCG: iterations within 1, residuals and
    solution."""
    n, p = 48, 3
    pl = I.Plan(2, n, p, precision="f32")
    r = workloads.uniform_rhs(2, n, p, seed=11)
    assert np.array_equal(host(pl.apply_noalloc(dev(r))), host(pl.apply(dev(r))))
    ns, ps, dl = (n, 32), (p, 2), ((1, 0), (1, 1))
    pg = I.Plan(2, list(ns), list(ps), precision="f32", dirichlet=list(dl))
    assert pg.route() == "dense2d"
    pre = G.GeneralPreconditioner([(nk, pk, DSET[dk]) for nk, pk, dk in zip(ns, ps, dl)], "iffd_b")
    f = workloads.uniform_tensor(pre.shape, seed=5)
    uo, ito, conv, *_ = krylov.pcg(pre.matvec, pre.apply, f, tol=1e-8)
    assert conv
    u, st = pg.solve(dev(f), rtol=1e-8, maxit=100)
    s = st[0]
    print("dense2d PCG iterations", s["iterations"], "oracle", ito, flush=True)
    assert s["converged"] and s["status"] == 0
    assert abs(s["iterations"] - ito) <= 1
    assert s["relres"] <= 1e-8 and s["relres_true"] <= 2e-8
    assert rel(host(u), uo) <= 1e-6
