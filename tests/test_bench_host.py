"""Host logic of bench.py (no GPU): the one-GPU contract, the algorithmic
byte model behind the roofline fraction, and the rule that the HBM traffic
counters are reported only when they were taken on the current kernel
sources."""

import importlib.util
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
_spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
bench = importlib.util.module_from_spec(_spec)
_spec.loader.exec_module(bench)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_algorithmic_bytes_per_apply():
    """Each pass reads and writes the tensor once: FP64 at the ends of the
    apply, the transform precision in between (48N in 3D and 32N in 2D with
    the FP32 apply, 16(2d-1)N in FP64)."""
    N = 1000
    assert sum(bench.pass_bytes(3, N, "f32")) == 48 * N
    assert sum(bench.pass_bytes(2, N, "f32")) == 32 * N
    for d in (2, 3):
        assert sum(bench.pass_bytes(d, N, "f64")) == 16 * (2 * d - 1) * N
    assert bench.pass_bytes(3, N, "f32") == [12 * N, 8 * N, 8 * N, 8 * N, 12 * N]
    assert bench.pass_names(3) == ["fwd_axis1", "fwd_axis2", "mid_axis3", "bwd_axis2",
                                   "bwd_axis1"]


def test_traffic_record_used_only_on_its_sources(monkeypatch):
    import paper_2512_20269_amd.profiling as prof
    path = os.path.join(ROOT, "profiles", "traffic_cube_n128_p3_f32.json")
    with open(path) as fh:
        recorded = json.load(fh)["source_hash"]
    monkeypatch.setattr(prof, "source_hash", lambda: recorded)
    t = bench.load_traffic("cube_n128_p3", "f32")
    assert t is not None and len(t["passes"]) == 5
    # every pass moves 1.00-1.10x its algorithmic bytes in the recorded counters
    for entry in t["passes"]:
        for v in entry.values():
            assert 1.0 <= v["ratio"] <= 1.1
    monkeypatch.setattr(prof, "source_hash", lambda: "0" * 16)
    assert bench.load_traffic("cube_n128_p3", "f32") is None
    assert bench.load_traffic("no_such_workload", "f32") is None


def test_percentile_helper():
    xs = [5.0, 1.0, 3.0, 2.0, 4.0]
    assert bench.pct(xs, 0.5) == 3.0
    assert bench.pct(xs, 0.99) == 5.0
    assert bench.pct(xs, 0.0) == 1.0
