"""Build the HIP library libiffd.so in-tree for gfx950.

    python paper_2512_20269_amd/build.py

(run as a script: importing the package would load the library being built)

Every source is compiled with hipcc (device code for gfx950 only) with
packed FP32 instructions disabled, then linked into one shared library next
to this file.  The sources compile in parallel; a full build takes about a
minute on 8 cores.
"""

from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libiffd.so")

SOURCES = ["plan.cpp", "api.cpp", "apply.hip",
           "apply_la_fwd.hip", "apply_la_bwd.hip", "apply_la_mid.hip",
           "apply_lb_fwd.hip", "apply_lb_bwd.hip", "apply_lb_mid.hip",
           "apply_lc_fwd.hip", "apply_lc_bwd.hip", "apply_lc_mid.hip",
           "apply_ld_fwd.hip", "apply_ld_bwd.hip", "apply_ld_mid.hip",
           "apply_le_fwd.hip", "apply_le_bwd.hip", "apply_le_mid.hip",
           "apply_lf_fwd.hip", "apply_lf_bwd.hip", "apply_lf_mid.hip",
           "apply_lg_fwd.hip", "apply_lg_bwd.hip", "apply_lg_mid.hip",
           "gen.hip", "gen_la.hip", "gen_lb.hip", "gen_lc.hip", "gen_ld.hip", "gen_le.hip",
           "gen_lf.hip", "gen_lg.hip",
           "setup.hip", "matvec.hip", "mvroll.hip", "geo.hip", "pcg.hip", "dense.hip", "dense2d.hip", "noalloc.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-result",
          f"--offload-arch={ARCH}",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          f"-I{os.path.join(HERE, '..', 'include')}"]


def _headers_mtime() -> float:
    hs = [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".h")]
    hs.append(os.path.join(HERE, "..", "include", "iffd.h"))
    return max(os.path.getmtime(h) for h in hs)


def _compile(src: str, changed_only: bool = False) -> str:
    obj = os.path.join(BUILD, src + ".o")
    if changed_only and os.path.exists(obj):
        newest = max(os.path.getmtime(os.path.join(CSRC, src)), _headers_mtime())
        if os.path.getmtime(obj) > newest:
            return obj
    cmd = [HIPCC] + COMMON + ["-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {src}\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = True, changed_only: bool = False) -> str:
    """Compile every source (changed_only: skip objects newer than their
    source and every header) and link the library."""
    os.makedirs(BUILD, exist_ok=True)
    jobs = min(len(SOURCES), max(1, min(16, os.cpu_count() or 1)))
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda f: _compile(f, changed_only), SOURCES))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", f"--offload-arch={ARCH}", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


def clean() -> None:
    shutil.rmtree(BUILD, ignore_errors=True)


if __name__ == "__main__":
    if len(sys.argv) > 1 and sys.argv[1] == "clean":
        clean()
    else:
        build(changed_only=len(sys.argv) > 1 and sys.argv[1] == "--changed")
