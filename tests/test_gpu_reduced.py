"""GPU parity of reduced regularity (Remark rmk:reduced_regularity,
eq:reg_space2: an interior breakpoint repeated mult times in some directions)
against oracle.reduced (route B, pinned against route A).  Tolerances as for
the general plans: FP64 apply 1e-12, FP32 apply 1e-5, FP64 operator 1e-13
(relative 2-norm, max-norm and boundary-slab RMS, test_gpu_parity.check);
PCG in FP64 takes the oracle's iterations.  The cases cover a C^0 knot
(mult = p) and intermediate continuity, odd and even degree, Dirichlet,
natural and mixed ends, the knot along direction 1 (contiguous lines), a
strided direction and the middle pass's direction, and lengths to 256."""

import functools

import numpy as np
import pytest

import workloads
from oracle import krylov
from oracle import reduced as R

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2512_20269_amd as I  # noqa: E402
from test_gpu_parity import check, dev, host, rel  # noqa: E402

TOL = {"f64": 1e-12, "f32": 1e-5}
DSET = {(1, 1): {0, 1}, (1, 0): {0}, (0, 1): {1}, (0, 0): set()}


def specs_of(n, p, dl, knots):
    return tuple((nk, pk, frozenset(DSET[tuple(dk)]), knots.get(k + 1))
                 for k, (nk, pk, dk) in enumerate(zip(n, p, dl)))


@functools.lru_cache(maxsize=None)
def red_oracle(specs):
    return R.ReducedPreconditioner([(n, p, set(D), kt) for n, p, D, kt in specs], "iffd_b")


def red_plan(n, p, dl, knots, prec):
    return I.Plan(len(n), list(n), list(p), precision=prec, dirichlet=[tuple(x) for x in dl],
                  knots=knots)


# (n, p, ends, {direction: (k, mult)})
CASES = [
    ((32, 24), (3, 2), ((1, 1), (1, 1)), {1: (16, 3)}),
    ((32, 24), (4, 3), ((1, 0), (0, 1)), {1: (13, 2)}),
    ((32, 24), (2, 4), ((0, 0), (1, 1)), {1: (12, 2)}),
    ((24, 32), (2, 5), ((0, 0), (1, 0)), {2: (16, 5)}),
    ((32, 24, 32), (3, 2, 4), ((1, 0), (0, 1), (0, 0)), {1: (16, 3), 3: (16, 4)}),
    ((48, 32, 32), (5, 3, 3), ((1, 1), (1, 1), (1, 1)), {2: (16, 2)}),
    ((128, 32), (3, 4), ((1, 1), (0, 1)), {1: (64, 3)}),
    ((256, 16), (6, 3), ((0, 1), (1, 1)), {1: (100, 4)}),
]


def case_id(c):
    n, p, dl, kn = c
    return f"n{n}-p{p}-k{sorted(kn.items())}".replace(" ", "")


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("n,p,dl,knots", CASES, ids=[case_id(c) for c in CASES])
def test_reduced_apply_matches_oracle(n, p, dl, knots, prec):
    pre = red_oracle(specs_of(n, p, dl, knots))
    pl = red_plan(n, p, dl, knots, prec)
    assert pl.shape == pre.shape
    r = workloads.uniform_tensor(pre.shape, seed=sum(n) + 7 * sum(p))
    print(f"reduced apply n={n} p={p} {dl} knots={knots} {prec}", flush=True)
    z = host(pl.apply(dev(r)))
    check(z, pre.apply(r), TOL[prec], len(n), max(p), f"reduced n={n} p={p} {knots} {prec}")


@pytest.mark.parametrize("n,p,dl,knots", CASES[:6], ids=[case_id(c) for c in CASES[:6]])
def test_reduced_matvec_matches_oracle(n, p, dl, knots):
    pre = red_oracle(specs_of(n, p, dl, knots))
    pl = red_plan(n, p, dl, knots, "f64")
    x = workloads.uniform_tensor(pre.shape, seed=5 + sum(n))
    y = host(pl.matvec(dev(x)))
    check(y, pre.matvec(x), 1e-13, len(n), max(p), f"reduced matvec n={n} {knots}")


def test_reduced_pcg_matches_oracle():
    """3D, C^0 knots in two directions: FP64 PCG takes the oracle's
    iterations; FP32 within one."""
    n, p, dl, knots = (32, 32, 32), (3, 3, 3), ((1, 0), (0, 1), (0, 0)), {1: (16, 3), 3: (12, 3)}
    pre = red_oracle(specs_of(n, p, dl, knots))
    f = workloads.uniform_tensor(pre.shape, seed=1)
    uo, ito, conv, *_ = krylov.pcg(pre.matvec, pre.apply, f, tol=1e-8)
    assert conv
    for prec in ("f64", "f32"):
        u, st = red_plan(n, p, dl, knots, prec).solve(dev(f), rtol=1e-8, maxit=100)
        s = st[0]
        print(prec, "iterations", s["iterations"], "oracle", ito, flush=True)
        assert s["converged"]
        assert abs(s["iterations"] - ito) <= (0 if prec == "f64" else 1)
        assert rel(host(u), uo) <= 1e-6


@pytest.mark.parametrize("n", [64, 128, 256])
def test_reduced_iterations_robust(n):
    """h- and p-robustness with a C^0 line (Table 5's setting on the cube):
    a C^0 knot at x_1 = 1/2 (mult = p) on the mixed cube of Table 3 takes at
    most two more IFFD iterations than maximal smoothness."""
    dl = workloads.MIXED_CUBE_DIRICHLET
    for p in (2, 3, 4, 5):
        f0 = workloads.uniform_tensor(red_plan((n,) * 3, (p,) * 3, dl, {}, "f32").shape, seed=1)
        _, s0 = red_plan((n,) * 3, (p,) * 3, dl, {}, "f32").solve(dev(f0), rtol=1e-8, maxit=100)
        pl = red_plan((n,) * 3, (p,) * 3, dl, {1: (n // 2, p)}, "f32")
        f = workloads.uniform_tensor(pl.shape, seed=1)
        _, st = pl.solve(dev(f), rtol=1e-8, maxit=100)
        print(f"n={n} p={p}: C^0 knot {st[0]['iterations']} smooth {s0[0]['iterations']}",
              flush=True)
        assert st[0]["converged"] and st[0]["iterations"] <= s0[0]["iterations"] + 2
        del pl
        torch.cuda.empty_cache()
