#!/usr/bin/env python3
"""Benchmark of the IFFD preconditioner apply on one MI355X.

    python bench.py [--steps K] [--warmup W] [--workload NAME] [--precision f32|f64]

A step is one application z = P^{-1} r of the FFT-based Fast Diagonalization
preconditioner (forward line transforms along every direction, Kronecker-sum
scaling, backward transforms) to the workload's right-hand sides, already
resident in HBM.  Default workload: 3D unit cube, n = 256 elements per
direction, degree p = 3 (16,974,593 DoFs, the largest single-GPU
configuration), smooth right-hand side, FP32 transform arithmetic with FP64
input and output.

The K timed steps are enqueued back to back behind a device-side spin (so the
host never starves the GPU) with a HIP event after every step; then every pass
kernel is launched K times back to back between two events, which gives its
average duration (the roofline figure).  The same apply replayed from a HIP
graph is timed as well.

Printed as one JSON line: apply throughput (GDoF/s) with the roofline of its
dominant kernel, the same apply in FP64, PCG solve latency to 1e-8 (FP64 PCG,
this apply), the dense-FD baseline (apply on the matrix cores and PCG), PCG
with both preconditioners on a variable-coefficient system matrix (c = 1 + x
per direction, where neither is exact), the serving stream (Poisson arrivals
of mixed solves at four fractions of saturation), and the FP64 CPU oracle
timed on the host cores (all cores and one thread), whose result also gives
the GPU applies' error against the oracle.
"""

from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFS = 78.6   # FP64 vector: 256 CUs x 64 FMA lanes per clock x 2 x 2.4 GHz
MFMA_PEAK_TFLOPS = {"f32": 157.3, "f64": 78.6}
METRIC = "FFT-FD apply GDoF/s vs dense FD; PCG solves/s + p99 latency to 1e-8 rel res"

# name: (d, n, p, right-hand sides, RHS recipe)
WORKLOADS = {
    "cube_n128_p3": (3, 128, 3, 1, "uniform[-1,1] seed 2"),
    "square_n64_p3": (2, 64, 3, 1, "uniform[-1,1] seed 1"),
    "cube_n256_p2": (3, 256, 2, 1, "smooth 8-mode sine + 1e-3 noise, seed 3"),
    "cube_n256_p3": (3, 256, 3, 1, "smooth 8-mode sine + 1e-3 noise, seed 3"),
    "cube_n256_p4": (3, 256, 4, 1, "smooth 8-mode sine + 1e-3 noise, seed 3"),
    "cube_n256_p6": (3, 256, 6, 1, "smooth 8-mode sine + 1e-3 noise, seed 3"),
    "cube_n256_p8": (3, 256, 8, 1, "smooth 8-mode sine + 1e-3 noise, seed 3"),
    "cube_n96_p4_b64": (3, 96, 4, 64, "uniform[-1,1], seeds 4000+b"),
}


def make_rhs(workload):
    import workloads
    if workload.startswith("cube_n256_p"):
        return workloads.workload_rhs("cube_n256", p=int(workload[len("cube_n256_p"):]))
    return workloads.workload_rhs(workload)


def pass_bytes(d, N, prec):
    """Algorithmic HBM bytes of each pass over one right-hand side: the
    tensor is read once and written once (FP64 at the ends of the apply,
    the transform precision in between)."""
    w = 8 if prec == "f64" else 4
    out = []
    for k in range(2 * d - 1):
        rd = 8 if k == 0 else w
        wr = 8 if k == 2 * d - 2 else w
        out.append(N * (rd + wr))
    return out


def pass_names(d):
    names = [f"fwd_axis{k + 1}" for k in range(d - 1)] + [f"mid_axis{d}"]
    names += [f"bwd_axis{k}" for k in range(d - 1, 0, -1)]
    return names


def load_traffic(workload, prec):
    """HBM bytes per dispatch measured with rocprofv3 counters, if they were
    taken on the current kernel sources (else None)."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}_{prec}.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        t = json.load(fh)
    from paper_2512_20269_amd.profiling import source_hash
    if t.get("source_hash") != source_hash():
        return None
    return t


def sleep_cycles_per_ms(torch):
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    torch.cuda._sleep(1_000_000)
    b.record()
    torch.cuda.synchronize()
    return 1_000_000 / max(a.elapsed_time(b), 1e-3)


def pct(xs, q):
    xs = sorted(xs)
    return xs[min(len(xs) - 1, int(q * len(xs)))]


def cpu_baseline(d, n, p, r_np, budget_s=12.0):
    """The FP64 oracle (dense O(m^2)-per-line mode products) on the host cores,
    applied to the first right-hand side: as many repetitions as fit the
    budget with all cores, then one with a single thread.  Returns the record
    and the oracle's result (for the GPU applies' error against it)."""
    from threadpoolctl import threadpool_info, threadpool_limits
    from oracle import iffd as O
    t0 = time.perf_counter()
    pre = O.Preconditioner(d, n, p, "iffd_b")
    t_setup = time.perf_counter() - t0
    t0 = time.perf_counter()
    zo = pre.apply(r_np)
    t1 = time.perf_counter() - t0
    reps = max(1, min(20, int(budget_s / max(t1, 1e-3))))
    ts = [t1]
    for _ in range(reps - 1):
        t0 = time.perf_counter()
        pre.apply(r_np)
        ts.append(time.perf_counter() - t0)
    dt = statistics.median(ts)
    with threadpool_limits(1):
        t0 = time.perf_counter()
        pre.apply(r_np)
        dt1 = time.perf_counter() - t0
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    N = r_np.size
    return {"value": round(N / dt / 1e9, 6), "unit": "GDoF/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{reps} FP64 oracle applies (structured route, dense mode products) "
                      f"of one {d}D n={n} p={p} right-hand side with all threads (median "
                      f"{dt * 1e3:.1f} ms), then one with a single thread",
            "ms_per_apply_all_threads": round(dt * 1e3, 2),
            "ms_per_apply_one_thread": round(dt1 * 1e3, 2),
            "single_thread_gdof_s": round(N / dt1 / 1e9, 6),
            "oracle_setup_s": round(t_setup, 2),
            "host_nproc": os.cpu_count(), "affinity_cpus": len(os.sched_getaffinity(0)),
            "omp_num_threads": os.environ.get("OMP_NUM_THREADS")}, zo


def time_solves(torch, plan, f, count, rtol=1e-8):
    u, st = plan.solve(f, rtol=rtol)
    torch.cuda.synchronize()
    lat = []
    for _ in range(count):
        t0 = time.perf_counter()
        u, st = plan.solve(f, rtol=rtol, out=u)
        torch.cuda.synchronize()
        lat.append((time.perf_counter() - t0) * 1e3)
    return lat, st


def serving(torch, count, warm, fracs, budget_gb=96.0, slots=8, iters=2, check=4):
    """Continuous-batching solve server on a Poisson stream of mixed (d, n, p)
    requests: a saturation run (every request present at t = 0) and one run
    per QPS = frac x saturation throughput.  Latency = arrival -> result."""
    import workloads
    import paper_2512_20269_amd as iffd
    from paper_2512_20269_amd.serve import Request, SolveServer
    spec = workloads.serving_requests(warm + count, qps=1.0)
    fs = [torch.from_numpy(workloads.uniform_rhs(d, n, p, rs)).cuda()
          for (_, d, n, p, rs) in spec]
    srv = SolveServer(int(budget_gb * 2**30), slots=slots, iters_per_round=iters)

    def reqs(ids, qps):
        t_first = spec[ids[0]][0]
        return [Request(k, 0.0 if qps is None else (spec[k][0] - t_first) / qps,
                        *spec[k][1:4], fs[k]) for k in ids]

    srv.run(reqs(list(range(warm)), None))          # warm the resident plans
    ids = list(range(warm, warm + count))

    def measure(qps):
        r0 = (srv.launches, srv.busy_slots_at_launch, srv.inflight_at_launch)
        done = [r for r in srv.run(reqs(ids, qps)) if r.status != "rejected"]
        lat = [(r.t_done - r.arrival) * 1e3 for r in done]
        span = max(r.t_done for r in done) - min(r.arrival for r in done)
        launches = srv.launches - r0[0]
        res = {"qps_offered": None if qps is None else round(qps, 2),
               "solves_per_s": round(len(done) / span, 2), "completed": len(done),
               "p50_ms": round(pct(lat, 0.5), 3), "p99_ms": round(pct(lat, 0.99), 3),
               "mean_slots_per_launch":
                   round((srv.busy_slots_at_launch - r0[1]) / max(launches, 1), 2),
               "mean_shapes_in_flight":
                   round((srv.inflight_at_launch - r0[2]) / max(launches, 1), 2),
               "all_converged": all(r.status == 0 for r in done)}
        buckets = {}
        for r in done:
            b = f"d{r.d}_n{'<=64' if r.n <= 64 else ('96-128' if r.n <= 128 else '192-256')}"
            buckets.setdefault(b, []).append((r.t_done - r.arrival) * 1e3)
        res["by_bucket"] = {b: {"count": len(v), "p50_ms": round(pct(v, 0.5), 3),
                                "p99_ms": round(pct(v, 0.99), 3)}
                            for b, v in sorted(buckets.items())}
        return res, done

    sat, done = measure(None)
    runs = []
    for frac in fracs:
        res, done = measure(frac * sat["solves_per_s"])
        res["frac_of_saturation"] = frac
        runs.append(res)
    # a request's solution is the same bits alone (its own single-slot plan)
    same = True
    for r in done[:: max(1, len(done) // check)][:check]:
        solo = iffd.Plan(r.d, r.n, r.p, method="fft", precision="f32", max_rhs=1)
        u1, _ = solo.solve(r.f, rtol=1e-8, maxit=200)
        same = same and bool(torch.equal(u1, r.u))
    return {"requests": count, "warmup_requests": warm, "slots_per_shape": slots,
            "iters_per_round": iters, "hbm_budget_gb": budget_gb,
            "peak_footprint_gb": round(srv.peak / 2**30, 2), "saturation": sat,
            "runs": runs, "sampled_same_bits_as_alone": same, "sampled": check}


def mixed_bc(torch, iffd, ps=(3,), n=256, steps=20, solves=10, prec="f32"):
    """Section 7's cube with mixed boundary conditions (Table 3: Dirichlet on
    x = 0 and y = 1, natural conditions elsewhere) through a general plan:
    apply throughput with per-pass durations and the roofline of the
    dominant pass, and PCG to 1e-8 (iterations against Table 3)."""
    import workloads
    cpm = sleep_cycles_per_ms(torch)
    rows = []
    for p in ps:
        pl = iffd.Plan(3, [n] * 3, [p] * 3, precision=prec,
                       dirichlet=workloads.MIXED_CUBE_DIRICHLET)
        N = pl.N
        f = torch.from_numpy(workloads.uniform_tensor(pl.shape, seed=1)).cuda()
        z = torch.empty_like(f)
        for _ in range(3):
            pl.apply(f, out=z)
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda._sleep(int(cpm * 5.0))
        a.record()
        for _ in range(steps):
            pl.apply(f, out=z)
        b.record()
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / steps
        npass = pl.n_passes()
        pp = []
        for k in range(npass):
            a_, b_ = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda._sleep(int(cpm * (2.0 + 0.03 * steps)))
            a_.record()
            for _ in range(steps):
                pl.apply_pass(k, f, z)
            b_.record()
            torch.cuda.synchronize()
            pp.append(a_.elapsed_time(b_) / steps)
        pb = pass_bytes(3, N, prec)
        names = pass_names(3)
        dom = max(range(npass), key=lambda k: pp[k])
        ach = pb[dom] / (pp[dom] * 1e-3) / 1e9
        lat, st = time_solves(torch, pl, f, solves)
        # the same preconditioner through a generic basis of S^reg
        # (eq:reg_eigenvectors: a banded interpolation solve per line)
        plg = iffd.Plan(3, [n] * 3, [p] * 3, precision=prec,
                        dirichlet=workloads.MIXED_CUBE_DIRICHLET, basis="generic")
        zg = torch.empty_like(f)
        for _ in range(3):
            plg.apply(f, out=zg)
        torch.cuda.synchronize()
        ag, bg = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda._sleep(int(cpm * 5.0))
        ag.record()
        for _ in range(steps):
            plg.apply(f, out=zg)
        bg.record()
        torch.cuda.synchronize()
        msg = ag.elapsed_time(bg) / steps
        pl.apply(f, out=z)
        gdiff = float(((zg - z).norm() / z.norm()).item())
        del plg, zg
        # reduced regularity: a C^0 plane x_1 = 1/2 (the breakpoint n/2 of
        # direction 1 repeated p times)
        plk = iffd.Plan(3, [n] * 3, [p] * 3, precision=prec,
                        dirichlet=workloads.MIXED_CUBE_DIRICHLET, knots={1: (n // 2, p)})
        fk = torch.from_numpy(workloads.uniform_tensor(plk.shape, seed=1)).cuda()
        zk = torch.empty_like(fk)
        for _ in range(3):
            plk.apply(fk, out=zk)
        torch.cuda.synchronize()
        torch.cuda._sleep(int(cpm * 5.0))
        ag.record()
        for _ in range(steps):
            plk.apply(fk, out=zk)
        bg.record()
        torch.cuda.synchronize()
        msk = ag.elapsed_time(bg) / steps
        latk, stk = time_solves(torch, plk, fk, solves)
        del plk, fk, zk
        # dense FD (every direction's exact eigendecomposition) on the same system
        pfd = iffd.Plan(3, [n] * 3, [p] * 3, method="dense", precision=prec,
                        dirichlet=workloads.MIXED_CUBE_DIRICHLET)
        zf = torch.empty_like(f)
        for _ in range(3):
            pfd.apply(f, out=zf)
        torch.cuda.synchronize()
        torch.cuda._sleep(int(cpm * 5.0))
        ag.record()
        for _ in range(steps):
            pfd.apply(f, out=zf)
        bg.record()
        torch.cuda.synchronize()
        apfd = ag.elapsed_time(bg) / steps
        latfd, stfd = time_solves(torch, pfd, f, solves)
        del pfd, zf
        rows.append({
            "n": n, "p": p, "shape": list(pl.shape), "dofs": N, "dtype": prec,
            "generic_basis": {"ms_per_apply": round(msg, 5),
                              "slowdown_vs_special": round(msg / ms, 3),
                              "rel_diff_vs_special": gdiff},
            "c0_plane": {"ms_per_apply": round(msk, 5),
                         "pcg_p50_ms": round(pct(latk, 0.5), 3),
                         "iterations": stk[0]["iterations"]},
            "gdof_s": round(N / (ms * 1e-3) / 1e9, 3), "ms_per_apply": round(ms, 5),
            "roofline": {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4),
                         "kernel": f"gen_line_pass {names[dom]}",
                         "alg_bytes_per_launch": pb[dom],
                         "per_pass_us": {names[k]: round(pp[k] * 1e3, 2) for k in range(npass)},
                         "apply_alg_GBs": round(sum(pb) / (ms * 1e-3) / 1e9, 1)},
            "pcg": {"solves_per_s": round(1e3 / statistics.mean(lat), 2),
                    "p50_ms": round(pct(lat, 0.5), 3), "p99_ms": round(pct(lat, 0.99), 3),
                    "iterations": st[0]["iterations"], "relres_true": st[0]["relres_true"]},
            "dense_fd": {"apply_us": round(apfd * 1e3, 2),
                         "pcg_p50_ms": round(pct(latfd, 0.5), 3),
                         "iterations": stfd[0]["iterations"],
                         "iffd_solve_speedup": round(statistics.mean(latfd) / statistics.mean(lat), 3)}})
        del pl, f, z
        torch.cuda.empty_cache()
    return rows


def geo_flops_per_element(p):
    """Algorithmic FP64 flops of the mapped-domain operator per element, P =
    p + 1: the sum factorization (forward and backward along three
    directions, 16 P^4 fused multiply-adds) plus about 50 flops per Gauss
    point for G and w G grad u."""
    P = p + 1
    return 32 * P ** 4 + 50 * P ** 3


def annulus(torch, iffd, ps=(3,), n=64, steps=20, solves=5, prec="f32"):
    """Section 7's thick quarter of annulus (Table 4: Dirichlet on the bottom
    face, natural conditions elsewhere): the mapped-domain operator
    (matrix-free, FP64) against the FP64 ALU peak, the IFFD apply, and PCG to
    1e-8 (iterations against Table 4)."""
    import workloads
    rows = []
    for p in ps:
        pl = iffd.Plan(3, [n] * 3, [p] * 3, precision=prec,
                       dirichlet=workloads.ANNULUS_DIRICHLET,
                       geometry=("annulus", workloads.ANNULUS_PARAMS))
        f = torch.from_numpy(workloads.uniform_tensor(pl.shape, seed=1)).cuda()
        z = torch.empty_like(f)

        def timed(fn):
            for _ in range(3):
                fn()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            a.record()
            for _ in range(steps):
                fn()
            b.record()
            torch.cuda.synchronize()
            return a.elapsed_time(b) / steps

        mv = timed(lambda: pl.matvec(f, out=z))
        ap = timed(lambda: pl.apply(f, out=z))
        lat, st = time_solves(torch, pl, f, solves)
        # dense FD (exact eigendecompositions) on the same system
        pfd = iffd.Plan(3, [n] * 3, [p] * 3, method="dense", precision=prec,
                        dirichlet=workloads.ANNULUS_DIRICHLET,
                        geometry=("annulus", workloads.ANNULUS_PARAMS))
        apfd = timed(lambda: pfd.apply(f, out=z))
        latfd, stfd = time_solves(torch, pfd, f, solves)
        del pfd
        flops = n ** 3 * geo_flops_per_element(p)
        ach = flops / (mv * 1e-3) / 1e12
        rows.append({
            "n": n, "p": p, "dofs": pl.N, "dtype": prec,
            "operator_us": round(mv * 1e3, 2), "apply_us": round(ap * 1e3, 2),
            "roofline": {"bound": "alu", "achieved": round(ach, 2), "peak": FP64_PEAK_TFS,
                         "unit": "TFLOP/s", "frac": round(ach / FP64_PEAK_TFS, 4),
                         "kernel": "geometry operator (geo_element_lines + geo_gather)",
                         "alg_flops_per_launch": flops},
            "pcg": {"solves_per_s": round(1e3 / statistics.mean(lat), 2),
                    "p50_ms": round(pct(lat, 0.5), 3), "p99_ms": round(pct(lat, 0.99), 3),
                    "iterations": st[0]["iterations"], "relres_true": st[0]["relres_true"]},
            "dense_fd": {"apply_us": round(apfd * 1e3, 2),
                         "pcg_p50_ms": round(pct(latfd, 0.5), 3),
                         "iterations": stfd[0]["iterations"],
                         "iffd_solve_speedup": round(statistics.mean(latfd) / statistics.mean(lat), 3)}})
        del pl, f, z
        torch.cuda.empty_cache()
    return rows


def plate(torch, iffd, d=3, ns=(32, 64, 128), ps=(2, 3, 4, 5), solves=3, prec="f32"):
    """The plate with a hole whose map is only C^0 across xi_1 = 1/2, on the
    space C^0 there too (the breakpoint n/2 of direction 1 repeated p times,
    Remark rmk:reduced_regularity): PCG to 1e-8 with IFFD and with dense FD
    (the stand-in for Table 5).  3D: extruded, Dirichlet on the bottom face;
    2D: the plate itself, Dirichlet on the whole boundary."""
    import workloads
    rows = []
    for n in ns:
        for p in ps:
            row = {"d": d, "n": n, "p": p}
            for method in ("fft", "dense"):
                pl = iffd.Plan(d, [n] * d, [p] * d, method=method, precision=prec,
                               dirichlet=(workloads.PLATE_DIRICHLET if d == 3
                                          else ((1, 1), (1, 1))),
                               knots={1: (n // 2, p)},
                               geometry=("plate", workloads.PLATE_PARAMS[:d]))
                f = torch.from_numpy(workloads.uniform_tensor(pl.shape, seed=1)).cuda()
                lat, st = time_solves(torch, pl, f, solves)
                row["dofs"] = pl.N
                row["iffd" if method == "fft" else "dense_fd"] = {
                    "iterations": st[0]["iterations"], "p50_ms": round(pct(lat, 0.5), 3),
                    "relres_true": st[0]["relres_true"]}
                del pl, f
                torch.cuda.empty_cache()
            rows.append(row)
    return rows


def small2d(torch, iffd, ns=(32, 64, 96), p=3, batches=(1, 16, 64, 256, 1024), inner=20,
            outer=10):
    """2D FP32 applies of small problems (uniform Dirichlet, p = 3), replayed
    from HIP graphs of `inner` applies each (so no host work per apply): the
    small 2-D route (dense Qt, two launches of LDS products) against the
    three line passes, per batch size, and the route the automatic choice
    takes for a plan of that batch capacity."""
    import workloads

    rows = []
    for n in ns:
        for b in batches:
            if n >= 96 and b > 256:
                continue
            pl = iffd.Plan(2, n, p, precision="f32", max_rhs=b)
            auto = pl.route(b)
            R = workloads.batched_uniform_rhs(2, n, p, list(range(b)))
            r = torch.from_numpy(R if b > 1 else R[0]).cuda()
            z = torch.empty_like(r)
            row = {"n": n, "p": p, "m": pl.shape[0], "nrhs": b, "auto": auto}
            for rt in ("dense2d", "passes"):
                pl.set_route(rt)
                cap = torch.cuda.Stream()
                cap.wait_stream(torch.cuda.current_stream())
                g = torch.cuda.CUDAGraph()
                with torch.cuda.stream(cap):
                    pl.apply(r, out=z)
                    torch.cuda.synchronize()
                    with torch.cuda.graph(g, stream=cap):
                        for _ in range(inner):
                            pl.apply(r, out=z)
                torch.cuda.current_stream().wait_stream(cap)
                g.replay()
                torch.cuda.synchronize()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                for _ in range(outer):
                    g.replay()
                e1.record()
                torch.cuda.synchronize()
                us = e0.elapsed_time(e1) * 1e3 / (inner * outer)
                row[rt + "_us"] = round(us, 2)
                row[rt + "_gdof_s"] = round(b * pl.shape[0] * pl.shape[1] / (us * 1e-6) / 1e9, 2)
            pl.set_route("auto")
            rows.append(row)
            print(json.dumps(row), file=sys.stderr, flush=True)
    return rows


def sweep_p(torch, ps=(2, 3, 4, 6, 8), n=256, coef=0.0):
    """3D with the smooth right-hand side (8 random-phase sine modes plus 1e-3
    noise, seed 3), degree sweep: FP32 apply error against the FP64 apply, PCG
    iterations and solve time with the FP32 apply, and the dense-FD solve
    beside it.  (The FP64 apply's agreement with the oracle is a GPU test.)
    coef != 0: the system matrix is A_c with c(x) = 1 + coef x per direction
    (both preconditioners stay those of A-hat, so neither is exact)."""
    import workloads
    import paper_2512_20269_amd as iffd
    rows = []
    for p in ps:
        f_np = workloads.smooth_rhs(3, n, p, 3)
        f = torch.from_numpy(f_np).cuda()
        row = {"n": n, "p": p, "coef_a": coef}
        p32 = iffd.Plan(3, n, p, method="fft", precision="f32", coef_a=coef)
        p32.tune(reps=5)
        z32 = p32.apply(f)
        z64 = iffd.Plan(3, n, p, method="fft", precision="f64").apply(f)
        row["apply_f32_relerr_vs_f64"] = float((z32 - z64).norm() / z64.norm())
        lat, st = time_solves(torch, p32, f, 5)
        u = p32.solve(f, rtol=1e-8)[0]
        row.update({"pcg_iterations": st[0]["iterations"], "pcg_relres_true": st[0]["relres_true"],
                    "pcg_ms_p50": round(pct(lat, 0.5), 3), "kappa_est": round(st[0]["kappa_est"], 4)})
        fd = iffd.Plan(3, n, p, method="dense", precision="f32", coef_a=coef)
        flat, fst = time_solves(torch, fd, f, 3)
        uf = fd.solve(f, rtol=1e-8)[0]
        row.update({"dense_fd_iterations": fst[0]["iterations"],
                    "dense_fd_ms_p50": round(pct(flat, 0.5), 3),
                    "solution_reldiff_iffd_vs_dense": float((u - uf).norm() / uf.norm())})
        rows.append(row)
        print(json.dumps(row), file=sys.stderr, flush=True)
        del p32, fd, z32, z64, u, uf
    return rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="cube_n256_p3", choices=sorted(WORKLOADS))
    ap.add_argument("--precision", default="f32", choices=["f32", "f64"])
    ap.add_argument("--solves", type=int, default=30)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="only the timed apply loop (for profiling)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="after the run, copy MIB MiB with a plain elementwise kernel "
                         "(reference dispatch for HBM byte counters)")
    ap.add_argument("--small2d", action="store_true",
                    help="only the small 2D applies (dense route vs line passes, graph-replayed)")
    ap.add_argument("--sweep-p", action="store_true",
                    help="only the 3D n=256 degree sweep (smooth right-hand side)")
    ap.add_argument("--sweep-n", default="",
                    help="only the IFFD / dense-FD solve comparison at these 3D sizes "
                         "(comma-separated n; p = 3 and 4, smooth right-hand side)")
    ap.add_argument("--coef", type=float, default=0.0,
                    help="solve with the variable-coefficient system matrix A_c, "
                         "c(x) = 1 + COEF x per direction (preconditioners of A-hat); the apply "
                         "does not depend on it")
    ap.add_argument("--serve", action="store_true",
                    help="only the serving benchmark (Poisson stream of mixed solves)")
    ap.add_argument("--pcg-only", choices=["fft", "dense"],
                    help="only PCG solves of the workload's first right-hand side with this "
                         "preconditioner (3 warm-up + --solves timed; for kernel traces)")
    ap.add_argument("--mixed", action="store_true",
                    help="only the mixed-boundary cube of Table 3 (n = 256, p = 2..5)")
    ap.add_argument("--annulus", action="store_true",
                    help="only the thick quarter of annulus of Table 4 (n = 64, p = 2..5)")
    ap.add_argument("--plate", action="store_true",
                    help="only the plate with a hole and a C^0 line: 2D n = 64, 128, 256 and "
                         "3D n = 32, 64, 128, p = 2..5")
    ap.add_argument("--serve-requests", type=int, default=1000)
    ap.add_argument("--serve-warmup", type=int, default=100)
    ap.add_argument("--serve-fracs", default="0.25,0.5,0.75,0.9")
    ap.add_argument("--serve-iters", type=int, default=2,
                    help="PCG iterations per shape and round of the solve server")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (one process, no collectives); "
              f"--gpus {args.gpus} is not supported", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2512_20269_amd as iffd

    torch.cuda.set_device(0)
    if args.sweep_n:
        rows = []
        for n_ in [int(x) for x in args.sweep_n.split(",")]:
            rows += sweep_p(torch, ps=(3, 4), n=n_, coef=args.coef)
        cs = f"_coef{args.coef:g}" if args.coef else ""
        print(json.dumps({"metric": "PCG solve time to 1e-8, IFFD vs dense FD", "unit": "ms",
                          "config": {"workload": f"cube_n{args.sweep_n}_p3-4_smooth{cs}"},
                          "rows": rows}), flush=True)
        return
    if args.sweep_p:
        rows = sweep_p(torch, coef=args.coef)
        cs = f"_coef{args.coef:g}" if args.coef else ""
        print(json.dumps({"metric": "iterations and FP32 apply error vs p, 3D n=256",
                          "n_gpus": 1, "dtype": "f32", "data": "synthetic",
                          "config": {"workload": f"cube_n256_p2-8_smooth{cs}"}, "rows": rows}),
              flush=True)
        return
    if args.mixed:
        rows = mixed_bc(torch, iffd, ps=(2, 3, 4, 5), steps=args.steps, solves=args.solves,
                        prec=args.precision)
        print(json.dumps({"metric": "mixed-boundary cube apply GDoF/s and PCG iterations",
                          "unit": "GDoF/s", "n_gpus": 1, "dtype": args.precision,
                          "data": "synthetic",
                          "config": {"workload": "mixed_cube_n256_p2-5_uniform"},
                          "rows": rows}), flush=True)
        return
    if args.annulus:
        rows = annulus(torch, iffd, ps=(2, 3, 4, 5), steps=args.steps, solves=args.solves,
                       prec=args.precision)
        print(json.dumps({"metric": "mapped-domain operator and PCG, thick quarter of annulus",
                          "unit": "ms", "n_gpus": 1, "dtype": args.precision,
                          "data": "synthetic",
                          "config": {"workload": "annulus_n64_p2-5_uniform"},
                          "rows": rows}), flush=True)
        return
    if args.small2d:
        rows = small2d(torch, iffd)
        print(json.dumps({"metric": "2D FP32 apply of small problems, graph-replayed", "unit": "us",
                          "n_gpus": 1, "dtype": "f32", "data": "synthetic",
                          "config": {"workload": "square_n32-96_p3_small"}, "rows": rows}))
        return
    if args.plate:
        rows = plate(torch, iffd, d=2, ns=(64, 128, 256), solves=args.solves,
                     prec=args.precision)
        rows += plate(torch, iffd, d=3, solves=args.solves, prec=args.precision)
        print(json.dumps({"metric": "PCG iterations and solve time, plate with a C^0 line "
                                    "(2D) or plane (3D)",
                          "unit": "ms", "n_gpus": 1, "dtype": args.precision,
                          "data": "synthetic",
                          "config": {"workload": "plate_c0_2d_n64-256_3d_n32-128_p2-5_uniform"},
                          "rows": rows}), flush=True)
        return
    if args.serve:
        res = serving(torch, args.serve_requests, args.serve_warmup,
                      [float(x) for x in args.serve_fracs.split(",")], iters=args.serve_iters)
        print(json.dumps({"metric": "PCG solves/s and p50/p99 latency, serving stream",
                          "unit": "solves/s", "value": res["saturation"]["solves_per_s"],
                          "n_gpus": 1, "higher_is_better": True, "dtype": "f32",
                          "data": "synthetic",
                          "config": {"workload": "serving_mixed_d2_3_n32_256_p2_6"},
                          "serving": res}), flush=True)
        return
    d, n, p, B, recipe = WORKLOADS[args.workload]
    if args.pcg_only:
        f_np = make_rhs(args.workload)
        f = torch.from_numpy(f_np[0] if B > 1 else f_np).cuda()
        pl = iffd.Plan(d, n, p, method=args.pcg_only, precision=args.precision,
                       coef_a=args.coef)
        if args.pcg_only == "fft":
            pl.tune(reps=20)
        for _ in range(2):
            pl.solve(f, rtol=1e-8)
        lat, st = time_solves(torch, pl, f, args.solves)
        print(json.dumps({"metric": "PCG solve to 1e-8 relative residual", "unit": "ms",
                          "value": round(statistics.mean(lat), 4), "higher_is_better": False,
                          "p50_ms": round(pct(lat, 0.5), 4), "p99_ms": round(pct(lat, 0.99), 4),
                          "iterations": st[0]["iterations"], "method": args.pcg_only,
                          "dtype": args.precision, "solves": args.solves, "coef_a": args.coef,
                          "config": {"workload": args.workload}}), flush=True)
        return
    r_np = make_rhs(args.workload)
    r = torch.from_numpy(r_np).cuda()
    z = torch.empty_like(r)
    # (coef_a changes only the system matrix of the solves, not the apply)
    plan = iffd.Plan(d, n, p, method="fft", precision=args.precision, max_rhs=B,
                     coef_a=args.coef)
    N = plan.N
    npass = plan.n_passes()
    variants = plan.tune(reps=20)   # FFT shape per pass, timed on the device

    for _ in range(max(args.warmup, 1)):
        plan.apply(r, out=z)
    torch.cuda.synchronize()

    # ---- timed region: K applies back to back, an event after every step -----
    cpm = sleep_cycles_per_ms(torch)
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    torch.cuda._sleep(int(cpm * (5.0 + 0.03 * args.steps * npass)))
    evs[0].record()
    for s in range(args.steps):
        plan.apply(r, out=z)
        evs[s + 1].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    total_ms = evs[0].elapsed_time(evs[-1])
    ms_per_step = total_ms / args.steps
    value = B * N / (ms_per_step * 1e-3) / 1e9
    # ---- each pass kernel's average duration: K launches of that pass back to
    # back between two events (no event between launches, so the span is the
    # kernels plus the dispatch gaps of a full queue) -------------------------
    per_pass = []
    for k in range(npass):
        a_, b_ = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda._sleep(int(cpm * (2.0 + 0.03 * args.steps)))
        a_.record()
        for s in range(args.steps):
            plan.apply_pass(k, r, z)
        b_.record()
        torch.cuda.synchronize()
        per_pass.append(a_.elapsed_time(b_) / args.steps)
    plan.apply(r, out=z)   # the passes above leave intermediate data in z and the workspace

    # ---- the same apply replayed from a HIP graph ------------------------------
    cap = torch.cuda.Stream()
    cap.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(cap):
        plan.apply(r, out=z)
        torch.cuda.synchronize()
        with torch.cuda.graph(g, stream=cap):
            plan.apply(r, out=z)
    torch.cuda.current_stream().wait_stream(cap)
    for _ in range(args.warmup):
        g.replay()
    torch.cuda.synchronize()
    g0, g1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda._sleep(int(cpm * 5.0))
    g0.record()
    for _ in range(args.steps):
        g.replay()
    g1.record()
    torch.cuda.synchronize()
    graph_ms = g0.elapsed_time(g1) / args.steps

    pb = [B * x for x in pass_bytes(d, N, args.precision)]
    names = pass_names(d)
    dom = max(range(npass), key=lambda k: per_pass[k])
    achieved = pb[dom] / (per_pass[dom] * 1e-3) / 1e9
    traffic = load_traffic(args.workload, args.precision)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": (traffic["passes"][dom][str(variants[dom])]["bytes"]
                            if traffic and str(variants[dom]) in traffic["passes"][dom]
                            else None),
                "kernel": f"line_pass {names[dom]}",
                "alg_bytes_per_launch": pb[dom],
                "per_pass_us": {names[k]: round(per_pass[k] * 1e3, 2) for k in range(npass)},
                "per_pass_alg_GBs": {names[k]: round(pb[k] / (per_pass[k] * 1e-3) / 1e9, 1)
                                     for k in range(npass)},
                "apply_alg_bytes": sum(pb),
                "apply_alg_GBs": round(sum(pb) / (ms_per_step * 1e-3) / 1e9, 1),
                "fft_len": plan.info["fft_len"], "fft_variant_per_pass": variants}
    if traffic:
        roofline["traffic_source"] = traffic["source"]

    out = {"metric": METRIC, "value": round(value, 3), "unit": "GDoF/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 5),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": args.precision, "data": "synthetic",
           "config": {"workload": args.workload, "d": d, "n": n, "p": p, "dofs_per_rhs": N,
                      "rhs": B, "rhs_recipe": recipe, "apply_io": "f64", "coef_a": args.coef,
                      "step": f"one preconditioner apply to {B} right-hand side(s)"},
           "graph_ms_per_step": round(graph_ms, 5),
           "graph_gdof_s": round(B * N / (graph_ms * 1e-3) / 1e9, 3),
           "wall_s_timed": round(wall, 4), "roofline": roofline}

    z64 = None
    if not args.no_extras:
        # ---- the same apply in FP64 arithmetic: throughput and its passes --------
        if args.precision == "f32":
            ref = iffd.Plan(d, n, p, method="fft", precision="f64", max_rhs=B)
            v64 = ref.tune(reps=10)
            z64 = ref.apply(r)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda._sleep(int(cpm * 5.0))
            e0.record()
            for _ in range(args.steps):
                ref.apply(r, out=z64)
            e1.record()
            torch.cuda.synchronize()
            ms64 = e0.elapsed_time(e1) / args.steps
            pp64 = []
            for k in range(npass):
                a_, b_ = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                torch.cuda._sleep(int(cpm * (2.0 + 0.03 * args.steps)))
                a_.record()
                for _ in range(args.steps):
                    ref.apply_pass(k, r, z64)
                b_.record()
                torch.cuda.synchronize()
                pp64.append(a_.elapsed_time(b_) / args.steps)
            ref.apply(r, out=z64)
            pb64 = [B * x for x in pass_bytes(d, N, "f64")]
            dom64 = max(range(npass), key=lambda k: pp64[k])
            ach64 = pb64[dom64] / (pp64[dom64] * 1e-3) / 1e9
            out["apply_f64"] = {
                "gdof_s": round(B * N / (ms64 * 1e-3) / 1e9, 3), "ms_per_apply": round(ms64, 5),
                "roofline": {"bound": "hbm", "achieved": round(ach64, 1), "peak": HBM_PEAK_GBS,
                             "unit": "GB/s", "frac": round(ach64 / HBM_PEAK_GBS, 4),
                             "kernel": f"line_pass {names[dom64]}",
                             "alg_bytes_per_launch": pb64[dom64],
                             "per_pass_us": {names[k]: round(pp64[k] * 1e3, 2)
                                             for k in range(npass)},
                             "apply_alg_GBs": round(sum(pb64) / (ms64 * 1e-3) / 1e9, 1)},
                "fft_variant_per_pass": v64}
            del ref
        # ---- accuracy of this apply against the FP64 apply -----------------------
        plan.apply(r, out=z)
        if z64 is not None:
            out["apply_relerr_vs_f64"] = float((z - z64).norm() / z64.norm())
        f = r[0] if B > 1 else r
        # ---- PCG solves to 1e-8 (FP64 PCG, this apply) ---------------------------
        lat, st = time_solves(torch, plan, f, args.solves)
        out["pcg"] = {"solves_per_s": round(1e3 / statistics.mean(lat), 2),
                      "p50_ms": round(pct(lat, 0.5), 3), "p99_ms": round(pct(lat, 0.99), 3),
                      "iterations": st[0]["iterations"], "relres_true": st[0]["relres_true"],
                      "kappa_est": round(st[0]["kappa_est"], 4), "solves": args.solves,
                      "rhs": "first right-hand side of the workload"}
        if B > 1:
            # ---- the whole batch: PCG with the iteration loop in a HIP graph ------
            gs = iffd.GraphSolver(plan, B, k=2)
            U, gst = gs.solve(r, rtol=1e-8)
            torch.cuda.synchronize()
            glat = []
            for _ in range(max(3, args.solves // 5)):
                t0 = time.perf_counter()
                U, gst = gs.solve(r, rtol=1e-8, out=U)
                torch.cuda.synchronize()
                glat.append((time.perf_counter() - t0) * 1e3)
            elat, est = time_solves(torch, plan, r, max(3, args.solves // 5))
            its = [s_["iterations"] for s_ in gst]
            out["batched_pcg"] = {
                "rhs": B, "graph_batch_ms_p50": round(pct(glat, 0.5), 3),
                "graph_batch_ms_p99": round(pct(glat, 0.99), 3),
                "graph_solves_per_s": round(B * 1e3 / statistics.mean(glat), 2),
                "eager_batch_ms_p50": round(pct(elat, 0.5), 3),
                "eager_solves_per_s": round(B * 1e3 / statistics.mean(elat), 2),
                "iterations_min_max": [min(its), max(its)],
                "all_converged": all(s_["converged"] for s_ in gst)}
            del gs, U
        # ---- dense FD baseline: apply on the matrix cores, and PCG ---------------
        try:
            fd = iffd.Plan(d, n, p, method="dense", precision=args.precision, max_rhs=B,
                           coef_a=args.coef)
            zf = torch.empty_like(r)
            for _ in range(5):
                fd.apply(r, out=zf)
            torch.cuda.synchronize()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            reps = 20
            torch.cuda._sleep(int(cpm * 5.0))
            a.record()
            for _ in range(reps):
                fd.apply(r, out=zf)
            b.record()
            torch.cuda.synchronize()
            fms = a.elapsed_time(b) / reps
            flops = B * 4 * d * fd.m ** (d + 1)
            tf = flops / (fms * 1e-3) / 1e12
            flat, fst = time_solves(torch, fd, f, max(5, args.solves // 3))
            if B > 1:
                fblat, fbst = time_solves(torch, fd, r, max(3, args.solves // 5))
            out["dense_fd"] = {
                "gdof_s": round(B * N / (fms * 1e-3) / 1e9, 3), "ms_per_apply": round(fms, 5),
                "roofline": {"bound": "mfma", "achieved": round(tf, 2),
                             "peak": MFMA_PEAK_TFLOPS[args.precision], "unit": "TFLOP/s",
                             "frac": round(tf / MFMA_PEAK_TFLOPS[args.precision], 4),
                             "flops_per_apply": flops},
                "iffd_apply_speedup": round(fms / ms_per_step, 3),
                "pcg": {"solves_per_s": round(1e3 / statistics.mean(flat), 2),
                        "p50_ms": round(pct(flat, 0.5), 3), "p99_ms": round(pct(flat, 0.99), 3),
                        "iterations": fst[0]["iterations"]},
                "iffd_solve_speedup": round(statistics.mean(flat) / statistics.mean(lat), 3)}
            if B > 1:
                out["dense_fd"]["batched_pcg"] = {
                    "rhs": B, "batch_ms_p50": round(pct(fblat, 0.5), 3),
                    "solves_per_s": round(B * 1e3 / statistics.mean(fblat), 2),
                    "iterations": fbst[0]["iterations"]}
            del fd, zf
            # ---- dense FD on the FP16 / BF16 matrix cores, per-line scaling ------
            ref = iffd.Plan(d, n, p, method="dense", precision="f64", max_rhs=B)
            zd64 = ref.apply(r)
            del ref
            for hp, mfma in (("f16s", "v_mfma_f32_32x32x16_f16"),
                             ("bf16s", "v_mfma_f32_32x32x16_bf16")):
                fh = iffd.Plan(d, n, p, method="dense", precision=hp, max_rhs=B,
                               coef_a=args.coef)
                zh = torch.empty_like(r)
                for _ in range(5):
                    fh.apply(r, out=zh)
                torch.cuda.synchronize()
                torch.cuda._sleep(int(cpm * 5.0))
                a.record()
                for _ in range(reps):
                    fh.apply(r, out=zh)
                b.record()
                torch.cuda.synchronize()
                hms = a.elapsed_time(b) / reps
                herr = float((zh - zd64).norm() / zd64.norm())
                hlat, hst = time_solves(torch, fh, f, max(5, args.solves // 3))
                htf = flops / (hms * 1e-3) / 1e12
                # the 16-bit mode products are bound by HBM, not the matrix
                # cores: each moves the FP32 tensor in and out plus its 16-bit
                # copy (a quantization sweep reads FP32 and writes 16 bits)
                hbytes = B * N * 2 * d * (4 + 2 + 2 + 4) + B * N * 8 * 2
                out[f"dense_fd_{hp}"] = {
                    "gdof_s": round(B * N / (hms * 1e-3) / 1e9, 3),
                    "ms_per_apply": round(hms, 5), "apply_relerr_vs_f64": herr,
                    "roofline": {"bound": "mfma", "achieved": round(htf, 2), "peak": 2500.0,
                                 "unit": "TFLOP/s", "frac": round(htf / 2500.0, 4),
                                 "hbm_GBs": round(hbytes / (hms * 1e-3) / 1e9, 1),
                                 "note": f"GEMMs on {mfma} plus one quantization sweep "
                                         "per mode product"},
                    "pcg": {"solves_per_s": round(1e3 / statistics.mean(hlat), 2),
                            "p50_ms": round(pct(hlat, 0.5), 3),
                            "iterations": hst[0]["iterations"]}}
                del fh, zh
            del zd64
        except iffd.IffdError as e:
            out["dense_fd"] = {"error": str(e)}
        if B == 1 and args.coef == 0.0:
            # ---- a system matrix neither preconditioner inverts: A_c with the
            # coefficient 1 + x per direction, IFFD and dense FD of A-hat ------
            pc = iffd.Plan(d, n, p, method="fft", precision=args.precision, coef_a=1.0)
            pc.tune(reps=5)
            clat, cst = time_solves(torch, pc, f, max(5, args.solves // 3))
            del pc
            fc = iffd.Plan(d, n, p, method="dense", precision=args.precision, coef_a=1.0)
            cflat, cfst = time_solves(torch, fc, f, max(5, args.solves // 3))
            del fc
            out["pcg_variable_coefficient"] = {
                "coef_a": 1.0,
                "iffd": {"solves_per_s": round(1e3 / statistics.mean(clat), 2),
                         "p50_ms": round(pct(clat, 0.5), 3), "p99_ms": round(pct(clat, 0.99), 3),
                         "iterations": cst[0]["iterations"]},
                "dense_fd": {"solves_per_s": round(1e3 / statistics.mean(cflat), 2),
                             "p50_ms": round(pct(cflat, 0.5), 3),
                             "p99_ms": round(pct(cflat, 0.99), 3),
                             "iterations": cfst[0]["iterations"]},
                "iffd_solve_speedup": round(statistics.mean(cflat) / statistics.mean(clat), 3)}
            out["serving"] = serving(torch, args.serve_requests, args.serve_warmup,
                                     [float(x) for x in args.serve_fracs.split(",")],
                                     iters=args.serve_iters)
            # ---- the mixed-boundary cube of Table 3 through a general plan ------
            out["mixed_bc"] = mixed_bc(torch, iffd, ps=(3,), n=256, steps=min(args.steps, 50),
                                       solves=max(5, args.solves // 3), prec=args.precision)[0]
            # ---- the mapped domain of Table 4 (thick quarter of annulus) --------
            out["annulus"] = annulus(torch, iffd, ps=(3,), n=64, steps=min(args.steps, 20),
                                     solves=max(3, args.solves // 5), prec=args.precision)[0]
            # ---- the plate with a C^0 line (Table 5's setting, 2D) -------------
            out["plate"] = plate(torch, iffd, d=2, ns=(256,), ps=(3,),
                                 solves=max(3, args.solves // 5), prec=args.precision)[0]
            # ---- small 2D problems: the dense route against the line passes ------
            out["small2d"] = small2d(torch, iffd, ns=(64,), batches=(1, 64, 1024))
    if args.copy_calibration > 0:
        nel = args.copy_calibration * (1 << 20) // 8
        src = torch.ones(nel, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            torch.neg(src, out=dst)
        torch.cuda.synchronize()
        out["copy_calibration_bytes"] = {"read": nel * 8, "write": nel * 8}
    if not args.no_cpu_baseline:
        r0 = r_np[0] if B > 1 else r_np
        out["cpu_baseline"], zo = cpu_baseline(d, n, p, r0)
        # the GPU applies against the oracle's result for the same input
        import numpy as np
        plan.apply(r, out=z)
        zs = {args.precision: (z[0] if B > 1 else z).cpu().numpy()}
        if z64 is not None:
            zs["f64"] = (z64[0] if B > 1 else z64).cpu().numpy()
        out["apply_error_vs_oracle"] = {
            k: {"rel_2norm": float(np.linalg.norm(v - zo) / np.linalg.norm(zo)),
                "rel_maxnorm": float(np.abs(v - zo).max() / np.abs(zo).max())}
            for k, v in zs.items()}
        out["apply_error_vs_oracle"]["tolerance"] = {"f32": 1e-5, "f64": 1e-12}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
