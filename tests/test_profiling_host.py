"""Host logic of the measurement tooling (paper_2512_20269_amd/profiling.py),
on synthetic rocprofv3 databases: the traffic record's calibration against a
copy kernel of known size, the per-pass byte ratios, the kernel-trace
summary, and the comment-insensitive source hash that decides whether a
traffic record still describes the kernels."""

import sqlite3

import pytest

from paper_2512_20269_amd import profiling as prof


def make_counter_db(path, counter, rows):
    c = sqlite3.connect(path)
    c.execute("create table counters_collection (kernel_name text, counter_name text, value real)")
    c.executemany("insert into counters_collection values (?, ?, ?)",
                  [(k, counter, v) for k, v in rows])
    c.commit()
    c.close()


def test_traffic_calibration_and_ratios(tmp_path):
    d, n, p, L, N = 3, 128, 3, 128, 129 ** 3
    names = [prof.line_pass_name(d, "f32", k, L, 4, n, p) for k in range(5)]
    alg = [N * 12, N * 8, N * 8, N * 8, N * 12]
    # the copy of 1 GiB reads half its bytes in FETCH_SIZE (factor 2) and all in WRITE_SIZE
    copy = "void at::native::neg_kernel(...)"
    fetch = [(copy, 1 << 19)] + [(nm + "(float const*)", a / 2 / 2 / 1024) for nm, a in zip(names, alg)]
    write = [(copy, 1 << 20)] + [(nm + "(float const*)", a / 2 / 1024) for nm, a in zip(names, alg)]
    # (each pass: half its bytes read, half written, FETCH seeing half of the reads)
    make_counter_db(tmp_path / "f.db", "FETCH_SIZE", fetch)
    make_counter_db(tmp_path / "w.db", "WRITE_SIZE", write)
    bench = {"copy_calibration_bytes": {"read": 1 << 30, "write": 1 << 30},
             "config": {"d": d, "dofs_per_rhs": N, "rhs": 1, "n": n, "p": p,
                        "workload": "cube_n128_p3"},
             "roofline": {"fft_variant_per_pass": [4] * 5, "fft_len": L}, "dtype": "f32"}
    t = prof.traffic(str(tmp_path / "f.db"), str(tmp_path / "w.db"), bench, "cf", "cw")
    assert t["copy_calibration"]["fetch_scale"] == pytest.approx(2.0)
    assert t["copy_calibration"]["write_scale"] == pytest.approx(1.0)
    assert [e["4"]["alg_bytes"] for e in t["passes"]] == alg
    for e in t["passes"]:
        assert e["4"]["ratio"] == pytest.approx(1.0, abs=1e-3)
    assert t["source_hash"] == prof.source_hash()


def test_kernel_trace_summary(tmp_path):
    c = sqlite3.connect(tmp_path / "k.db")
    c.execute("create table kernels (name text, duration real)")
    c.executemany("insert into kernels values (?, ?)",
                  [("void iffd::a<1>(int)", 3000.0), ("void iffd::a<1>(int)", 1000.0),
                   ("iffd::b(double*)", 6000.0)])
    c.commit()
    c.close()
    text = prof.stats_text(str(tmp_path / "k.db"), "cmd")
    rows = [ln for ln in text.splitlines() if ln.startswith("| `")]
    assert rows[0].startswith("| `iffd::b(double*)` | 1 | 6.00 |")     # sorted by total
    assert rows[1].startswith("| `void iffd::a<1>` | 2 | 2.00 | 1.00 | 3.00 | 4.0 | 40.0 |")


def test_source_hash_ignores_comments_only():
    code = "int f(int x) {  // a note\n  return x + 1; /* more */\n}\n"
    assert prof._code_only(code) == prof._code_only(
        "int f(int x) {  // another note\n  return x + 1;\n}\n")
    assert prof._code_only(code) != prof._code_only("int f(int x) {\n  return x + 2;\n}\n")
