"""GPU parity of general plans (per-direction n, p and Dirichlet / natural
ends: Section 4 "other boundary conditions", Table 1, Section 6) against the
oracle's general route (oracle/general.py: special basis of eq:special_basis,
the explicit sine / cosine matrices of Table 1, eigenvalues as seminorm
quotients).  Tolerances as for the Dirichlet plans: FP64 apply 1e-12, FP32
apply 1e-5, FP64 operator 1e-13, each as a relative 2-norm, a max-norm and a
boundary-slab RMS (see test_gpu_parity.check).  The cases cover the eight
transforms of Table 1 (four end-condition sets times odd / even degree),
anisotropic (n_k, p_k), the smallest n for a degree, p = 1, and the Table 3
experiment."""

import functools
import json
import os

import numpy as np
import pytest

import workloads
from oracle import general as G
from oracle import krylov

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2512_20269_amd as I  # noqa: E402
from test_gpu_parity import check, dev, host, oracle, plan, rel  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
TOL = {"f64": 1e-12, "f32": 1e-5}
DSET = {(1, 1): {0, 1}, (1, 0): {0}, (0, 1): {1}, (0, 0): set()}


def specs_of(n, p, dl):
    return tuple((nk, pk, frozenset(DSET[tuple(dk)])) for nk, pk, dk in zip(n, p, dl))


@functools.lru_cache(maxsize=None)
def gen_oracle(specs):
    return G.GeneralPreconditioner([(n, p, set(D)) for n, p, D in specs], "iffd_b")


@functools.lru_cache(maxsize=None)
def gen_plan(n, p, dl, prec="f32", max_rhs=1):
    return I.Plan(len(n), list(n), list(p), precision=prec, max_rhs=max_rhs,
                  dirichlet=[tuple(x) for x in dl])


# (n per direction, p per direction, (Dirichlet at 0, at 1) per direction)
CASES = [
    # the eight transforms of Table 1 along direction 1 (odd and even p)
    ((16, 24), (3, 3), ((1, 0), (1, 1))),
    ((16, 24), (4, 2), ((1, 0), (1, 1))),
    ((16, 24), (3, 3), ((0, 1), (1, 1))),
    ((16, 24), (4, 2), ((0, 1), (1, 1))),
    ((16, 24), (3, 3), ((0, 0), (1, 1))),
    ((16, 24), (4, 2), ((0, 0), (1, 1))),
    ((16, 24), (3, 3), ((1, 1), (0, 0))),
    ((16, 24), (2, 4), ((1, 1), (1, 0))),
    # the Table 3 pattern in 3D, anisotropic sizes and degrees
    ((16, 24, 32), (3, 2, 4), ((1, 0), (0, 1), (0, 0))),
    ((32, 16, 24), (5, 6, 3), ((0, 0), (1, 0), (0, 1))),
    ((24, 32, 16), (2, 3, 5), ((0, 1), (0, 0), (1, 1))),
    # high degrees at small n (the two end blocks nearly meet), p = 1
    ((12, 16), (7, 8), ((0, 0), (1, 0))),
    ((16, 12), (8, 7), ((0, 1), (0, 0))),
    ((16, 32), (1, 1), ((0, 0), (1, 0))),
    ((8, 16, 8), (1, 2, 7), ((1, 0), (0, 1), (0, 0))),
    # several tiles with ragged tails, the larger lengths
    ((96, 64), (3, 4), ((0, 1), (1, 0))),
    ((192, 48), (2, 5), ((1, 0), (0, 0))),
    ((256, 24), (4, 3), ((0, 0), (0, 1))),
    ((64, 64, 64), (3, 3, 3), ((1, 0), (0, 1), (0, 0))),
]


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("n,p,dl", CASES)
def test_general_apply_matches_oracle(n, p, dl, prec):
    pre = gen_oracle(specs_of(n, p, dl))
    pl = gen_plan(n, p, dl, prec)
    assert pl.shape == pre.shape
    r = workloads.uniform_tensor(pre.shape, seed=sum(n) + 10 * sum(p))
    print(f"general apply n={n} p={p} dirichlet={dl} {prec}", flush=True)
    z = host(pl.apply(dev(r)))
    check(z, pre.apply(r), TOL[prec], len(n), max(p), f"n={n} p={p} {dl} {prec}")


@pytest.mark.parametrize("n,p,dl", [c for c in CASES if len(c[0]) == 3] + CASES[:4])
def test_general_matvec_matches_oracle(n, p, dl):
    pre = gen_oracle(specs_of(n, p, dl))
    pl = gen_plan(n, p, dl, "f64")
    x = workloads.uniform_tensor(pre.shape, seed=7 + sum(n))
    print(f"general matvec n={n} p={p} dirichlet={dl}", flush=True)
    y = host(pl.matvec(dev(x)))
    check(y, pre.matvec(x), 1e-13, len(n), max(p), "matvec")


def test_general_dirichlet_equals_uniform_plan():
    """A general plan with Dirichlet ends everywhere and equal (n, p) is the
    preconditioner of the uniform plan (another route: length-2n transforms
    with twists instead of the tuned DST kernels); both within the FP64 gate
    of the oracle, so within 2e-12 of each other."""
    for d, n, p in [(3, 32, 3), (2, 64, 4), (3, 24, 6)]:
        r = workloads.uniform_rhs(d, n, p, seed=33 + n)
        zg = host(gen_plan((n,) * d, (p,) * d, ((1, 1),) * d, "f64").apply(dev(r)))
        zu = host(plan(d, n, p, "f64").apply(dev(r)))
        assert rel(zg, zu) <= 2e-12, (d, n, p, rel(zg, zu))
        check(zg, oracle(d, n, p).apply(r), 1e-12, d, p, f"dirichlet general d={d} n={n} p={p}")


def test_general_batch_equals_single_bitwise():
    n, p, dl = (24, 16, 32), (3, 4, 2), ((1, 0), (0, 1), (0, 0))
    pl = gen_plan(n, p, dl, "f32", max_rhs=3)
    shape = pl.shape
    R = np.stack([workloads.uniform_tensor(shape, seed=s) for s in (1, 2, 3)])
    Z = host(pl.apply(dev(R)))
    for b in range(3):
        z1 = host(pl.apply(dev(R[b])))
        assert np.array_equal(Z[b], z1)


def test_general_pcg_matches_oracle():
    """PCG on the Table 3 pattern (3D, n = 32, p = 3) against the oracle's PCG:
    iterations (FP64 apply: equal; FP32: within 1), residuals and solution."""
    n, p, dl = (32, 32, 32), (3, 3, 3), workloads.MIXED_CUBE_DIRICHLET
    pre = gen_oracle(specs_of(n, p, dl))
    f = workloads.uniform_tensor(pre.shape, seed=1)
    uo, ito, conv, *_ = krylov.pcg(pre.matvec, pre.apply, f, tol=1e-8)
    assert conv
    for prec in ("f64", "f32"):
        u, st = gen_plan(n, p, dl, prec).solve(dev(f), rtol=1e-8, maxit=100)
        s = st[0]
        print(prec, "iterations", s["iterations"], "oracle", ito, flush=True)
        assert s["converged"] and s["status"] == 0
        assert abs(s["iterations"] - ito) <= (0 if prec == "f64" else 1)
        assert s["relres"] <= 1e-8 and s["relres_true"] <= 2e-8
        assert rel(host(u), uo) <= 1e-6


@pytest.mark.parametrize("n", [64, 128, 256])
def test_table3_counts_on_gpu(n):
    """Table 3 (3D cube, Dirichlet on x = 0 and y = 1, natural elsewhere):
    PCG iterations with the FP32 apply within +-1 of the printed counts for
    p = 2..5 at n = 64, 128, 256 (tests/golden/table3_cube.json)."""
    g = json.load(open(os.path.join(HERE, "golden", "table3_cube.json")))
    printed = g["iterations"][g["n"].index(n)]
    dl = workloads.MIXED_CUBE_DIRICHLET
    for p, it_p in zip(g["p"], printed):
        pl = I.Plan(3, [n] * 3, [p] * 3, precision="f32", dirichlet=dl)
        f = workloads.uniform_tensor(pl.shape, seed=1)
        _, st = pl.solve(dev(f), rtol=1e-8, maxit=100)
        s = st[0]
        print(f"Table 3 n={n} p={p}: {s['iterations']} (printed {it_p})", flush=True)
        assert s["converged"] and abs(s["iterations"] - it_p) <= 1
        del pl
        torch.cuda.empty_cache()


def test_general_stepped_pcg_alone_equals_in_mix():
    """Stepped PCG on a general plan: a slot's iterate is the same alone and
    next to other solves (no cross-slot reduction)."""
    n, p, dl = (24, 32, 16), (3, 2, 4), ((0, 1), (1, 0), (0, 0))
    pl = gen_plan(n, p, dl, "f32", max_rhs=3)
    F = [workloads.uniform_tensor(pl.shape, seed=s) for s in (5, 6, 7)]
    one = I.PcgState(pl, 1)
    one.begin([0], dev(F[0]))
    mix = I.PcgState(pl, 3)
    mix.begin([0, 1, 2], dev(np.stack(F)))
    for _ in range(30):
        one.iterate(1)
        mix.iterate(1)
    a = host(one.take(0))
    b = host(mix.take(0))
    assert np.array_equal(a, b)
    st = mix.poll()
    assert st.shape == (3, 4)


def test_general_noalloc_equals_apply():
    n, p, dl = (32, 24, 16), (4, 3, 5), ((1, 0), (0, 0), (0, 1))
    pl = gen_plan(n, p, dl, "f32")
    r = dev(workloads.uniform_tensor(pl.shape, seed=9))
    assert torch.equal(pl.apply(r), pl.apply_noalloc(r))


# ---- the generic basis of eq:reg_eigenvectors (Q_reg = C^{-1} U D^{-1}) -------

@functools.lru_cache(maxsize=None)
def generic_oracle(specs):
    return G.GeneralPreconditioner([(n, p, set(D)) for n, p, D in specs], "iffd_generic")


@functools.lru_cache(maxsize=None)
def generic_plan(n, p, dl, prec="f32"):
    return I.Plan(len(n), list(n), list(p), precision=prec,
                  dirichlet=[tuple(x) for x in dl], basis="generic")


GENERIC_CASES = [
    # the eight transforms of Table 1 along direction 1 (odd and even p)
    ((16, 24), (3, 3), ((1, 0), (1, 1))),
    ((16, 24), (4, 2), ((1, 0), (1, 1))),
    ((16, 24), (3, 3), ((0, 1), (1, 1))),
    ((16, 24), (4, 2), ((0, 1), (1, 1))),
    ((16, 24), (3, 3), ((0, 0), (1, 1))),
    ((16, 24), (4, 2), ((0, 0), (1, 1))),
    ((16, 24), (5, 3), ((1, 1), (0, 0))),
    ((16, 24), (2, 4), ((1, 1), (1, 0))),
    # 3D mixed, the highest degrees, p = 1, several tiles with ragged tails
    ((16, 24, 32), (3, 2, 4), ((1, 0), (0, 1), (0, 0))),
    ((12, 16), (7, 8), ((0, 0), (1, 0))),
    ((16, 12), (8, 7), ((0, 1), (0, 0))),
    ((16, 32), (1, 1), ((0, 0), (1, 0))),
    ((96, 64), (3, 4), ((0, 1), (1, 0))),
    ((256, 24), (4, 3), ((0, 0), (0, 1))),
    ((64, 64, 64), (3, 3, 3), ((1, 0), (0, 1), (0, 0))),
]


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("n,p,dl", GENERIC_CASES)
def test_generic_basis_apply_matches_oracle(n, p, dl, prec):
    """The generic-basis plan (banded interpolation solves per line) against
    the oracle's generic route, which equals route B: P^{-1} r does not depend
    on the basis of S^reg."""
    pre = generic_oracle(specs_of(n, p, dl))
    pl = generic_plan(n, p, dl, prec)
    assert pl.shape == pre.shape
    r = workloads.uniform_tensor(pre.shape, seed=sum(n) + 10 * sum(p) + 1)
    print(f"generic-basis apply n={n} p={p} dirichlet={dl} {prec}", flush=True)
    z = host(pl.apply(dev(r)))
    check(z, pre.apply(r), TOL[prec], len(n), max(p), f"generic n={n} p={p} {dl} {prec}")


def test_generic_basis_pcg_equals_special():
    """PCG on the Table 3 pattern (3D, n = 32, p = 2..5) with both bases: the
    same preconditioner, so the same iterations (FP64 apply) and solutions."""
    n, dl = (32, 32, 32), workloads.MIXED_CUBE_DIRICHLET
    for p in (2, 3, 4, 5):
        f = workloads.uniform_tensor(gen_plan(n, (p,) * 3, dl, "f64").shape, seed=1)
        us, sts = gen_plan(n, (p,) * 3, dl, "f64").solve(dev(f), rtol=1e-8, maxit=100)
        ug, stg = generic_plan(n, (p,) * 3, dl, "f64").solve(dev(f), rtol=1e-8, maxit=100)
        print(f"p={p}: special {sts[0]['iterations']} generic {stg[0]['iterations']}", flush=True)
        assert stg[0]["converged"] and stg[0]["iterations"] == sts[0]["iterations"]
        assert rel(host(ug), host(us)) <= 1e-9


# ---- dense FD on general plans (each direction its own Q_k, Lambda_k) --------

FD_CASES = [CASES[0], CASES[3], CASES[4], CASES[8], CASES[9], CASES[12], CASES[15], CASES[18]]


@functools.lru_cache(maxsize=None)
def fd_oracle(specs):
    return G.GeneralPreconditioner([(n, p, set(D)) for n, p, D in specs], "fd")


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("n,p,dl", FD_CASES)
def test_general_dense_fd_matches_oracle(n, p, dl, prec):
    """Classical FD (eq:exact_diagonalization) with per-direction sizes and
    ends: the matrix-core mode products and the Kronecker-sum scaling against
    the oracle's dense FD."""
    pre = fd_oracle(specs_of(n, p, dl))
    pl = I.Plan(len(n), list(n), list(p), method="dense", precision=prec,
                dirichlet=[tuple(x) for x in dl])
    r = workloads.uniform_tensor(pre.shape, seed=sum(n) + 3)
    z = host(pl.apply(dev(r)))
    check(z, pre.apply(r), TOL[prec], len(n), max(p), f"general FD n={n} p={p} {dl} {prec}")


def test_general_dense_fd_with_a_repeated_knot():
    from oracle import reduced as Rd
    n, p, dl, kn = (32, 24), (3, 2), ((1, 0), (0, 1)), {1: (16, 3)}
    pre = Rd.ReducedPreconditioner([(32, 3, {0}, (16, 3)), (24, 2, {1}, None)], "fd")
    pl = I.Plan(2, list(n), list(p), method="dense", precision="f64",
                dirichlet=[tuple(x) for x in dl], knots=kn)
    r = workloads.uniform_tensor(pre.shape, seed=9)
    check(host(pl.apply(dev(r))), pre.apply(r), 1e-12, 2, 3, "FD with a repeated knot")
