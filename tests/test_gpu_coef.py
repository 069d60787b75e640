"""GPU parity for the variable-coefficient system matrix A_c
(iffd_opts.coef_a, c(x) = 1 + a x in every direction): the operator against
the oracle's, and PCG on A_c with the constant-coefficient preconditioners
(IFFD and dense FD, both built from A-hat) against the oracle's PCG with the
same preconditioner.  The paper prints no variable-coefficient counts that
need no geometry data, so the PCG comparison is oracle-only (parity
unpinned by the paper); A_c itself is pinned in test_oracle_coef.py."""

import functools

import numpy as np
import pytest

import workloads
from oracle import iffd as O
from oracle import krylov
from oracle import operator as OP

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2512_20269_amd as I  # noqa: E402


def rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def host(x):
    torch.cuda.synchronize()
    return x.cpu().numpy()


@functools.lru_cache(maxsize=None)
def operator(d, n, p, a):
    return OP.Operator(d, n, p, a)


@pytest.mark.parametrize("d,n,p,a", [(3, 48, 3, 1.0), (3, 32, 4, 4.0), (3, 24, 6, 1.0),
                                     (2, 64, 3, -0.5), (3, 16, 2, 2.0)])
def test_matvec_with_coefficient(d, n, p, a):
    """3D p <= 4 runs the fused operator (every band row distinct, so no
    tile takes the Toeplitz shortcut), p = 6 and 2D the two-pass one."""
    print(f"matvec coef d={d} n={n} p={p} a={a}", flush=True)
    x = workloads.uniform_rhs(d, n, p, seed=11 + n)
    pl = I.Plan(d, n, p, precision="f64", coef_a=a)
    y = host(pl.matvec(dev(x)))
    yo = operator(d, n, p, a).matvec(x)
    assert rel(y, yo) <= 1e-13


@pytest.mark.parametrize("d,n,p,a,method,prec", [
    (2, 64, 3, 1.0, "fft", "f64"), (2, 64, 3, 1.0, "dense", "f64"),
    (3, 24, 4, 3.0, "fft", "f32"), (3, 24, 4, 3.0, "dense", "f32"),
    (3, 16, 3, -0.5, "fft", "f32")])
def test_pcg_with_coefficient(d, n, p, a, method, prec):
    print(f"pcg coef d={d} n={n} p={p} a={a} {method} {prec}", flush=True)
    f = workloads.uniform_rhs(d, n, p, seed=21 + n)
    pre = O.Preconditioner(d, n, p, "iffd_b" if method == "fft" else "fd")
    uo, ito, conv, *_ = krylov.pcg(operator(d, n, p, a).matvec, pre.apply, f, tol=1e-8)
    assert conv
    u, st = I.Plan(d, n, p, method=method, precision=prec, coef_a=a).solve(dev(f), rtol=1e-8,
                                                                         maxit=200)
    s = st[0]
    assert s["converged"] and s["status"] == 0
    assert abs(s["iterations"] - ito) <= 1
    assert s["relres_true"] <= 2e-8
    assert rel(host(u), uo) <= 1e-6
    # FD of A-hat is no longer exact for A_c
    assert s["iterations"] > 2


@pytest.mark.parametrize("method", ["fft", "dense"])
def test_coefficient_batch_solves_equal_single_bitwise(method):
    """With the variable coefficient, a right-hand side solved in a batch of
    five gives the same bits and iterations as solved alone (per-slot tiles
    and fixed-order reductions; the operator's band tables are shared)."""
    d, n, p, a = 3, 16, 4, 2.0
    print(f"coef batch d={d} n={n} p={p} a={a} {method}", flush=True)
    R = workloads.batched_uniform_rhs(d, n, p, [41, 42, 43, 44, 45])
    plb = I.Plan(d, n, p, method=method, precision="f32", max_rhs=5, coef_a=a)
    U, stb = plb.solve(dev(R), rtol=1e-8, maxit=200)
    U = host(U)
    pl1 = I.Plan(d, n, p, method=method, precision="f32", max_rhs=1, coef_a=a)
    for k in (0, 2, 4):
        u1, st1 = pl1.solve(dev(R[k]), rtol=1e-8, maxit=200)
        assert np.array_equal(host(u1), U[k])
        assert st1[0]["iterations"] == stb[k]["iterations"]
