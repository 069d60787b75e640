"""Summaries of rocprofv3 output databases (rocpd SQLite) for the profiles/
folder: per-kernel duration statistics, and HBM bytes per dispatch of the
apply's line passes from the FETCH_SIZE / WRITE_SIZE counters.

    python -m paper_2512_20269_amd.profiling stats DB --cmd "..." [--out FILE]
    python -m paper_2512_20269_amd.profiling traffic --fetch DB1 --write DB2 \\
        --bench-json RUN.json --cmd-fetch "..." --cmd-write "..." [--out FILE]

The counters are reported in KiB per dispatch by the profiler and do not
necessarily cover every memory channel, so `traffic` scales them by what the
same counters read for a plain elementwise copy of known size dispatched in
the same run (bench.py --copy-calibration): scale = copy bytes / counter bytes.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sqlite3
import sys

HERE = os.path.dirname(os.path.abspath(__file__))


def _code_only(text: str) -> str:
    """C++ source without comments and whitespace (what the compiler sees)."""
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return re.sub(r"\s+", "", text)


def source_hash() -> str:
    """Hash of the line-pass kernel sources (code only; comments do not count);
    traffic measured on other code is stale."""
    h = hashlib.sha256()
    for f in ("apply_impl.h", "fft_device.h", "launch.h"):
        with open(os.path.join(HERE, "csrc", f)) as fh:
            h.update(_code_only(fh.read()).encode())
    return h.hexdigest()[:16]


def kernel_stats(db: str):
    """[(name, calls, total_ns, avg_ns, min_ns, max_ns)] sorted by total time."""
    c = sqlite3.connect(db)
    rows = c.execute("select name, count(*), sum(duration), avg(duration), min(duration), "
                     "max(duration) from kernels group by name order by 3 desc").fetchall()
    c.close()
    return rows


def counter_per_dispatch(db: str, counter: str):
    """{kernel name: (dispatches, mean counter value per dispatch)}."""
    c = sqlite3.connect(db)
    rows = c.execute("select kernel_name, count(*), avg(value) from counters_collection "
                     "where counter_name = ? group by kernel_name", (counter,)).fetchall()
    c.close()
    return {r[0]: (r[1], r[2]) for r in rows}


def short(name: str, width: int = 96) -> str:
    name = name.split("(")[0] if name.startswith("void ") else name
    return name if len(name) <= width else name[:width - 3] + "..."


def stats_text(db: str, cmd: str, top: int = 25) -> str:
    rows = kernel_stats(db)
    tot = sum(r[2] for r in rows) or 1
    out = [f"# rocprofv3 kernel trace summary", "", "Command:", "", "```", cmd, "```", "",
           "| kernel | calls | avg us | min us | max us | total us | % |",
           "|---|---:|---:|---:|---:|---:|---:|"]
    for name, calls, total, avg, mn, mx in rows[:top]:
        out.append(f"| `{short(name)}` | {calls} | {avg / 1e3:.2f} | {mn / 1e3:.2f} | "
                   f"{mx / 1e3:.2f} | {total / 1e3:.1f} | {100 * total / tot:.1f} |")
    return "\n".join(out) + "\n"


def line_pass_name(d: int, prec: str, k: int, L: int, variant: int, n: int, p: int) -> str:
    """Demangled name of pass k's kernel (see launch_iffd_pass); the last
    template argument is the sine-transform route (length n or 2n, parity)."""
    t = "double" if prec == "f64" else "float"
    tin = "double" if k == 0 else t
    if k == 0 and p >= 5:
        t = "double"   # FP32 plans of degree >= 5 take the FP64 input into an FP64 first pass
    tout = "double" if k == 2 * d - 2 else t
    mode = 0 if k < d - 1 else (2 if k == d - 1 else 1)
    route = (3 if p % 2 else 2) if L == n else (0 if p % 2 else 1)
    return f"void iffd::line_pass<{tin}, {tout}, {t}, {mode}, {L}, {variant}, {route}>"


def copy_entry(table):
    for name, v in table.items():
        if "neg" in name.lower():
            return v
    raise SystemExit("no calibration copy kernel in the profile (run bench.py with "
                     "--copy-calibration)")


def traffic(fetch_db: str, write_db: str, bench: dict, cmd_fetch: str, cmd_write: str) -> dict:
    fe = counter_per_dispatch(fetch_db, "FETCH_SIZE")
    wr = counter_per_dispatch(write_db, "WRITE_SIZE")
    cb = bench["copy_calibration_bytes"]
    f_copy, w_copy = copy_entry(fe)[1], copy_entry(wr)[1]
    fs = cb["read"] / (f_copy * 1024.0)
    ws = cb["write"] / (w_copy * 1024.0)
    cfg, roof = bench["config"], bench["roofline"]
    d, N, B, n, p = cfg["d"], cfg["dofs_per_rhs"], cfg["rhs"], cfg["n"], cfg["p"]
    prec = bench["dtype"]
    passes = []
    w = 8 if prec == "f64" else 4
    for k in range(len(roof["fft_variant_per_pass"])):
        alg = B * N * ((8 if k == 0 else w) + (8 if k == 2 * d - 2 else w))
        entry = {}
        for v in (0, 1, 2, 3, 4):    # the tuner dispatches every FFT shape of every pass
            name = line_pass_name(d, prec, k, roof["fft_len"], v, n, p)
            fk = [val for key, val in fe.items() if key.startswith(name + "(")]
            wk = [val for key, val in wr.items() if key.startswith(name + "(")]
            if not fk or not wk:
                continue
            fk, wk = fk[0][1], wk[0][1]
            entry[str(v)] = {"kernel": name, "fetch_kib": round(fk, 1),
                             "write_kib": round(wk, 1),
                             "bytes": int(fk * 1024 * fs + wk * 1024 * ws), "alg_bytes": alg,
                             "ratio": round((fk * 1024 * fs + wk * 1024 * ws) / alg, 3)}
        if not entry:
            raise SystemExit(f"pass {k}: no counters")
        passes.append(entry)
    return {"workload": cfg["workload"], "precision": prec, "source_hash": source_hash(),
            "source": "rocprofv3 --pmc FETCH_SIZE and --pmc WRITE_SIZE runs, scaled by an "
                      "elementwise copy of known size",
            "commands": [cmd_fetch, cmd_write],
            "copy_calibration": {"bytes_read": cb["read"], "bytes_written": cb["write"],
                                 "fetch_kib": round(f_copy, 1), "write_kib": round(w_copy, 1),
                                 "fetch_scale": round(fs, 4), "write_scale": round(ws, 4)},
            "passes": passes}


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="what", required=True)
    s = sub.add_parser("stats")
    s.add_argument("db")
    s.add_argument("--cmd", required=True)
    s.add_argument("--out")
    t = sub.add_parser("traffic")
    t.add_argument("--fetch", required=True)
    t.add_argument("--write", required=True)
    t.add_argument("--bench-json", required=True)
    t.add_argument("--cmd-fetch", required=True)
    t.add_argument("--cmd-write", required=True)
    t.add_argument("--out")
    a = ap.parse_args(argv)
    if a.what == "stats":
        text = stats_text(a.db, a.cmd)
    else:
        with open(a.bench_json) as fh:
            bench = json.loads([ln for ln in fh if ln.startswith("{")][-1])
        text = json.dumps(traffic(a.fetch, a.write, bench, a.cmd_fetch, a.cmd_write), indent=1)
    if a.out:
        with open(a.out, "w") as fh:
            fh.write(text)
    else:
        sys.stdout.write(text)


if __name__ == "__main__":
    main()
