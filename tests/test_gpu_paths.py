"""The plan kinds added on top of the Dirichlet and general plans (a mapped
domain's system matrix, a repeated knot, the generic basis) on the batched,
graph-replayed and stepped PCG paths: a batch member's solve equals its
single-RHS solve bit for bit, the HIP-graph replay equals the eager solve bit
for bit over repeated solves with eager work in between, and a stepped slot
gives the same bits alone and next to other solves."""

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2512_20269_amd as I  # noqa: E402
from test_gpu_parity import dev, host  # noqa: E402

B = 3


def make(kind):
    if kind == "annulus":
        return I.Plan(3, [16] * 3, [3] * 3, precision="f32", max_rhs=B,
                      dirichlet=workloads.ANNULUS_DIRICHLET,
                      geometry=("annulus", workloads.ANNULUS_PARAMS))
    if kind == "bump":
        return I.Plan(3, 16, 3, precision="f32", max_rhs=B, geometry=("bump", (0.05,)))
    if kind == "knot":
        return I.Plan(3, [32] * 3, [3] * 3, precision="f32", max_rhs=B,
                      dirichlet=workloads.MIXED_CUBE_DIRICHLET, knots={1: (16, 3)})
    if kind == "generic":
        return I.Plan(3, [32, 24, 16], [3, 2, 4], precision="f32", max_rhs=B,
                      dirichlet=[(1, 0), (0, 1), (0, 0)], basis="generic")
    raise ValueError(kind)


KINDS = ["annulus", "bump", "knot", "generic"]


@pytest.mark.parametrize("kind", KINDS)
def test_batch_graph_and_stepped_paths(kind):
    pl = make(kind)
    F = np.stack([workloads.uniform_tensor(pl.shape, seed=40 + b) for b in range(B)])
    Fd = dev(F)
    U, st = pl.solve(Fd, rtol=1e-8, maxit=200)
    U = host(U)
    assert all(s["converged"] for s in st), st
    for b in range(B):
        u1, s1 = pl.solve(dev(F[b]), rtol=1e-8, maxit=200)
        assert np.array_equal(U[b], host(u1)) and s1[0]["iterations"] == st[b]["iterations"]
    gs = I.GraphSolver(pl, B, k=1)
    for _ in range(2):
        ug, stg = gs.solve(Fd, rtol=1e-8, maxit=200)
        ug = host(ug)
        pl.apply(Fd)                  # unrelated eager work between the replays
        assert np.array_equal(ug, U)
        assert [s["iterations"] for s in stg] == [s["iterations"] for s in st]
    one = I.PcgState(pl, 1)
    one.begin([0], dev(F[1]))
    mix = I.PcgState(pl, B)
    mix.begin(list(range(B)), Fd)
    for _ in range(6):
        one.iterate(1)
        mix.iterate(1)
    assert np.array_equal(host(one.take(0)), host(mix.take(1)))
    print(f"{kind}: iterations {[s['iterations'] for s in st]}", flush=True)
