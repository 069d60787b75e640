"""The continuous-batching solve server: every request's solution is the
same bits as the same solve run alone, admission respects the HBM budget,
requests that cannot fit are rejected, idle shapes are evicted."""

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2512_20269_amd as I  # noqa: E402
from paper_2512_20269_amd.serve import Request, SolveServer  # noqa: E402


def make(spec):
    return [Request(k, t, d, n, p, torch.from_numpy(workloads.uniform_rhs(d, n, p, s)).cuda())
            for k, (t, d, n, p, s) in enumerate(spec)]


def solo(r):
    pl = I.Plan(r.d, r.n, r.p, method="fft", precision="f32", max_rhs=1)
    u, st = pl.solve(r.f, rtol=1e-8, maxit=200)
    return u, st[0]


def test_mixed_stream_same_bits_as_alone():
    spec = workloads.serving_requests(24, qps=400.0, seed=11, ns=(16, 24, 32), ps=(2, 3, 4, 5))
    reqs = make(spec)
    srv = SolveServer(8 * 2**30, slots=4, iters_per_round=2)
    done = srv.run(reqs)
    assert len(done) == len(reqs) and not srv.rejected
    assert srv.peak <= srv.budget
    for r in done:
        assert r.status == 0 and r.t_done >= r.arrival
        u, st = solo(r)
        assert torch.equal(u, r.u), (r.rid, r.key)
        assert st["iterations"] == r.iterations
    # several shapes were in flight together at some point
    assert srv.inflight_at_launch > srv.launches


def test_admission_budget_serializes_and_rejects():
    key = (3, 24, 3)
    need, N = SolveServer.entry_bytes(key, 2)
    budget = need + 8 * N            # the entry plus one result buffer
    spec = [(0.0, 3, 24, 3, 900 + k) for k in range(3)] + [(0.0, 3, 48, 3, 950)]
    reqs = make(spec)
    srv = SolveServer(budget, slots=2, iters_per_round=3)
    done = srv.run(reqs)
    assert [r.rid for r in srv.rejected] == [3]          # n = 48 cannot fit at all
    ok = [r for r in done if r.status != "rejected"]
    assert len(ok) == 3 and srv.peak <= budget
    # one at a time: each admitted after the previous one finished
    ok.sort(key=lambda r: r.t_admit)
    for a, b in zip(ok, ok[1:]):
        assert b.t_admit >= a.t_done
    for r in ok:
        u, _ = solo(r)
        assert torch.equal(u, r.u)


def test_idle_shapes_are_evicted():
    a, b = (2, 32, 3), (2, 32, 4)
    na, Na = SolveServer.entry_bytes(a, 2)
    nb, Nb = SolveServer.entry_bytes(b, 2)
    budget = max(na, nb) + 8 * max(Na, Nb)   # room for one shape at a time
    spec = [(0.0, *a, 1000), (0.0, *b, 1001), (0.0, *a, 1002)]
    srv = SolveServer(budget, slots=2, iters_per_round=2)
    done = srv.run(make(spec))
    assert all(r.status == 0 for r in done) and len(done) == 3
    assert srv.peak <= budget and len(srv.entries) == 1
    for r in done:
        u, _ = solo(r)
        assert torch.equal(u, r.u)


def test_graph_rounds_match_kernel_by_kernel_rounds():
    """A round replayed from the shape's HIP graph gives the same bits as the
    same round launched kernel by kernel, across replays with eager work in
    between (the server polls and copies between rounds)."""
    spec = workloads.serving_requests(10, qps=300.0, seed=13, ns=(16, 32), ps=(3, 4))
    out = []
    for graphs in (False, True):
        srv = SolveServer(8 * 2**30, slots=4, iters_per_round=2, graphs=graphs)
        done = sorted(srv.run(make(spec)), key=lambda r: r.rid)
        assert all(r.status == 0 for r in done)
        out.append(done)
    for a, b in zip(*out):
        assert torch.equal(a.u, b.u) and a.iterations == b.iterations
