#!/usr/bin/env python3
"""Benchmark of the IFFD preconditioner apply on one MI355X.

    python bench.py [--steps K] [--warmup W] [--workload NAME]

A step is one application z = P^{-1} r of the FFT-based Fast Diagonalization
preconditioner (forward line transforms along every direction, Kronecker-sum
scaling, backward transforms) to one right-hand side already resident in
HBM, in the default workload: 3D unit cube, n = 128 elements per direction,
degree p = 3 (2,146,689 DoFs), FP32 transform arithmetic with FP64 input and
output.  The K timed steps are replays of a HIP graph holding one apply.

Printed as one JSON line: the apply throughput (GDoF/s) with the roofline of
its dominant kernel (HIP events around each pass inside the timed loop), PCG
solve latency to 1e-8 (FP64 PCG, FP32 apply), the dense-FD baseline apply, and
the FP64 CPU oracle timed on the host cores on a bounded sample.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "FFT-FD apply GDoF/s vs dense FD; PCG solves/s + p99 latency to 1e-8 rel res"

WORKLOADS = {
    "cube_n128_p3": (3, 128, 3),
    "square_n64_p3": (2, 64, 3),
    "cube_n256_p3": (3, 256, 3),
    "cube_n96_p4": (3, 96, 4),
}


def pass_bytes(d, N, prec):
    """Algorithmic HBM bytes of each pass (read + write of the tensor once)."""
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


def source_hash():
    h = hashlib.sha256()
    for f in ("apply_impl.h", "fft_device.h"):
        with open(os.path.join(ROOT, "paper_2512_20269_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(workload, prec):
    """HBM bytes per dispatch measured with rocprofv3 counters, if they were
    taken on the current kernel sources (else None)."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}_{prec}.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        t = json.load(fh)
    if t.get("source_hash") != source_hash():
        return None
    return t


def sleep_cycles_for(torch, ms):
    """Cycles for torch.cuda._sleep to keep the GPU busy ~ms (lets the host
    enqueue a timed loop ahead of the device)."""
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    torch.cuda._sleep(1_000_000)
    b.record()
    torch.cuda.synchronize()
    per = max(a.elapsed_time(b), 1e-3) / 1_000_000
    return int(ms / per)


def cpu_baseline(d, n, p, r_np, budget_s=12.0):
    """The FP64 oracle (dense mode products) on the host cores."""
    from threadpoolctl import threadpool_info
    from oracle import iffd as O
    pre = O.Preconditioner(d, n, p, "iffd_b")
    t0 = time.perf_counter()
    pre.apply(r_np)
    t1 = time.perf_counter() - t0
    reps = max(1, min(20, int(budget_s / max(t1, 1e-3))))
    t0 = time.perf_counter()
    for _ in range(reps):
        pre.apply(r_np)
    dt = (time.perf_counter() - t0) / reps
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    N = r_np.size
    return {"value": round(N / dt / 1e9, 6), "unit": "GDoF/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{reps} FP64 oracle applies (dense O(m^2)-per-line mode products, "
                      f"structured route) of the same {d}D n={n} p={p} right-hand side; "
                      f"{dt * 1e3:.1f} ms per apply"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="cube_n128_p3", choices=sorted(WORKLOADS))
    ap.add_argument("--precision", default="f32", choices=["f32", "f64"])
    ap.add_argument("--solves", type=int, default=30)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="only the timed apply loop (for profiling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (one process, no collectives); "
              f"--gpus {args.gpus} is not supported", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2512_20269_amd as iffd
    import workloads

    d, n, p = WORKLOADS[args.workload]
    torch.cuda.set_device(0)
    if args.workload == "cube_n96_p4":
        r_np = workloads.uniform_rhs(d, n, p, seed=4000)
    elif args.workload in workloads.WORKLOADS:
        r_np = workloads.workload_rhs(args.workload)
    else:
        r_np = workloads.uniform_rhs(d, n, p, seed=2)
    r = torch.from_numpy(r_np).cuda()
    z = torch.empty_like(r)
    plan = iffd.Plan(d, n, p, method="fft", precision=args.precision)
    N = plan.N
    npass = plan.n_passes()
    variants = plan.tune(reps=20)   # FFT shape per pass, timed on the device

    # ---- warmup, then capture one apply in a HIP graph ----------------------
    for _ in range(max(args.warmup, 1)):
        plan.apply(r, out=z)
    torch.cuda.synchronize()
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

    # ---- timed region: K graph replays -----------------------------------------
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    e0.record()
    for _ in range(args.steps):
        g.replay()
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    ms_per_step = e0.elapsed_time(e1) / args.steps
    value = N / (ms_per_step * 1e-3) / 1e9

    # ---- per-kernel durations: HIP events between the passes ------------------
    cyc = sleep_cycles_for(torch, 30.0)
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(npass + 1)]
           for _ in range(args.steps)]
    torch.cuda._sleep(cyc)  # the host enqueues the loop while the GPU is busy
    for s in range(args.steps):
        evs[s][0].record()
        for k in range(npass):
            plan.apply_pass(k, r, z)
            evs[s][k + 1].record()
    torch.cuda.synchronize()
    per_pass = [statistics.mean(evs[s][k].elapsed_time(evs[s][k + 1]) for s in range(args.steps))
                for k in range(npass)]
    pb = pass_bytes(d, N, args.precision)
    names = pass_names(d)
    dom = max(range(npass), key=lambda k: per_pass[k])
    achieved = pb[dom] / (per_pass[dom] * 1e-3) / 1e9
    traffic = load_traffic(args.workload, args.precision)
    roofline = {"bound": "hbm", "kernel": f"line_pass {names[dom]}",
                "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic["passes"][dom] if traffic else None,
                "per_pass_us": {names[k]: round(per_pass[k] * 1e3, 2) for k in range(npass)},
                "per_pass_alg_GBs": {names[k]: round(pb[k] / (per_pass[k] * 1e-3) / 1e9, 1)
                                     for k in range(npass)},
                "apply_alg_bytes": sum(pb),
                "apply_alg_GBs": round(sum(pb) / (ms_per_step * 1e-3) / 1e9, 1),
                "fft_variant_per_pass": variants}

    out = {"metric": METRIC, "value": round(value, 3), "unit": "GDoF/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 5),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": args.precision, "data": "synthetic",
           "config": {"workload": args.workload, "d": d, "n": n, "p": p, "dofs": N,
                      "rhs": "uniform[-1,1] seed 2", "apply_io": "f64",
                      "step": "one preconditioner apply (HIP graph replay)"},
           "wall_s_timed": round(wall, 4), "roofline": roofline}

    if not args.no_extras:
        # ---- PCG solves to 1e-8 (FP64 PCG, this apply) ---------------------------
        lat, its = [], []
        u, st = plan.solve(r, rtol=1e-8)
        torch.cuda.synchronize()
        for _ in range(args.solves):
            t0 = time.perf_counter()
            u, st = plan.solve(r, rtol=1e-8, out=u)
            torch.cuda.synchronize()
            lat.append((time.perf_counter() - t0) * 1e3)
            its.append(st[0]["iterations"])
        lat.sort()
        out["pcg"] = {"solves_per_s": round(1e3 / statistics.mean(lat), 2),
                      "p50_ms": round(lat[len(lat) // 2], 3),
                      "p99_ms": round(lat[min(len(lat) - 1, int(0.99 * len(lat)))], 3),
                      "iterations": its[0], "relres_true": st[0]["relres_true"],
                      "kappa_est": round(st[0]["kappa_est"], 4), "solves": args.solves}
        # ---- dense FD baseline apply ---------------------------------------------
        try:
            fd = iffd.Plan(d, n, p, method="dense", precision=args.precision)
            zf = torch.empty_like(r)
            for _ in range(5):
                fd.apply(r, out=zf)
            torch.cuda.synchronize()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            for _ in range(50):
                fd.apply(r, out=zf)
            b.record()
            torch.cuda.synchronize()
            fms = a.elapsed_time(b) / 50
            flops = 4 * d * fd.m ** (d + 1)
            out["dense_fd"] = {"gdof_s": round(N / (fms * 1e-3) / 1e9, 3), "ms": round(fms, 5),
                               "tflops": round(flops / (fms * 1e-3) / 1e12, 2),
                               "iffd_speedup": round(fms / ms_per_step, 3)}
        except iffd.IffdError as e:
            out["dense_fd"] = {"error": str(e)}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(d, n, p, r_np)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
