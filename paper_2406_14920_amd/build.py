"""Builds libmdjk.so (gfx950) in-tree from csrc/ with hipcc.

    python -m paper_2406_14920_amd.build [--jobs N]

Every translation unit is compiled in parallel into _build/, then linked.
All HIP code is built with packed FP32 disabled.
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(os.path.dirname(HERE), "_build")
LIB = os.path.join(HERE, "libmdjk.so")

SOURCES = ["jeng_reg_0.hip", "jeng_reg_1.hip", "jeng_reg_2.hip", "jeng_reg_3.hip", "jeng_reg_q_0.hip",
           "jeng_reg_q_1.hip", "jeng_reg_q_2.hip", "jeng_reg_q_3.hip", "k_pair_6.hip", "k_small.hip", "k_wave_0.hip",
           "k_wave_1.hip", "k_wave_2.hip", "k_wave_3.hip", "k_wave_4.hip", "k_wave_5.hip", "k_pair_0.hip",
           "k_pair_1.hip", "k_pair_2.hip", "k_pair_3.hip", "k_pair_4.hip", "k_pair_5.hip", "k_pair_7.hip",
           "eprod.hip", "jeng.hip", "kg_0.hip", "kg_1.hip", "kg_2.hip", "kg_3.hip", "grad.hip", "setup.hip",
           "count.hip", "potential.hip", "grid.hip", "api.cpp"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-munsafe-fp-atomics",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wno-unused-result"]


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC] + FLAGS + ["-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
    t = time.time()
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s" % (" ".join(cmd), r.stderr[-6000:]))
    return "%s %.1fs" % (src, time.time() - t)


def _deps(path: str, seen: set) -> set:
    """The file and every quoted #include it reaches."""
    if path in seen or not os.path.exists(path):
        return seen
    seen.add(path)
    for line in open(path):
        line = line.strip()
        if line.startswith("#include \""):
            inc = line.split('"')[1]
            _deps(os.path.normpath(os.path.join(os.path.dirname(path), inc)), seen)
    return seen


def _stale(src: str) -> bool:
    """Object older than its source or one of the headers it includes."""
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    if not os.path.exists(obj):
        return True
    t = os.path.getmtime(obj)
    return any(os.path.getmtime(d) > t for d in _deps(os.path.join(CSRC, src), set()))


def build(jobs: int | None = None, verbose: bool = True, changed_only: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    if shutil.which(HIPCC) is None and not os.path.exists(HIPCC):
        raise RuntimeError("hipcc not found at %s" % HIPCC)
    jobs = jobs or min(16, os.cpu_count() or 4)
    t0 = time.time()
    todo = [s for s in SOURCES if _stale(s)] if changed_only else SOURCES
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        for msg in ex.map(_compile, todo):
            if verbose:
                print("  built", msg, flush=True)
    objs = [os.path.join(BUILD, os.path.splitext(s)[0] + ".o") for s in SOURCES]
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed: %s\n%s" % (" ".join(cmd), r.stderr[-4000:]))
    os.replace(tmp, LIB)
    if verbose:
        print("libmdjk.so linked in %.1fs total" % (time.time() - t0), flush=True)
    return LIB


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=None)
    ap.add_argument("--changed", action="store_true",
                    help="recompile only objects older than their source or a header")
    a = ap.parse_args()
    try:
        build(a.jobs, changed_only=a.changed)
    except RuntimeError as e:
        print(e, file=sys.stderr)
        sys.exit(1)
