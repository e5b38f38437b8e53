"""Build libetd.so (gfx950) from csrc/*.hip with hipcc, in-tree.

    python -m paper_2606_04347_amd.build [--jobs N] [--debug]

Every source is compiled to an object in _build/ (in parallel; fused.hip in
eight parts), then linked
into paper_2606_04347_amd/libetd.so.  Packed FP32 instructions are disabled
for all device code.
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libetd.so")
ARCH = os.environ.get("ETD_OFFLOAD_ARCH", "gfx950")

SOURCES = ["fft.hip", "fused.hip", "coupled.hip", "reduce.hip", "fixed.hip", "band.hip", "api.hip", "schedule.hip", "surface.hip"]
# (source, object name, extra flags): fused.hip is compiled in eight parts,
# each instantiating one pipeline in one precision, so they build in parallel
UNITS = [(s, os.path.splitext(s)[0], []) for s in SOURCES if s != "fused.hip"] + \
        [("fused.hip", f"fused{k}", [f"-DETD_FUSED_PART={k}"]) for k in range(8)]


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def flags(debug: bool):
    f = ["-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-I", INCLUDE, "-I", CSRC,
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         # multiply-adds fused only within one source expression, so a kernel
         # body rounds alike in its one-instance and its grouped form
         "-ffp-contract=on",
         "-Wall", "-Wno-unused-function", "-Wno-unused-variable"]
    f += ["-O1", "-g"] if debug else ["-O3"]
    return f


def compile_one(unit, debug: bool) -> str:
    src, name, extra = unit
    obj = os.path.join(BUILD, name + ".o")
    cmd = [hipcc(), *flags(debug), *extra, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    warn = "\n".join(l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l and l.strip())
    if warn and os.environ.get("ETD_BUILD_VERBOSE"):
        print(warn, file=sys.stderr)
    return obj


def build(jobs: int | None = None, debug: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    jobs = jobs or min(len(UNITS), max(1, (os.cpu_count() or 2)))
    # the eight fused parts first: they take longest
    order = sorted(UNITS, key=lambda u: u[0] != "fused.hip")
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda u: compile_one(u, debug), order))
    tmp = LIB + ".tmp"
    # roctx: the ranges around the stages of a step
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-lrocprofiler-sdk-roctx", "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=None)
    ap.add_argument("--debug", action="store_true")
    a = ap.parse_args()
    print(build(a.jobs, a.debug))


if __name__ == "__main__":
    main()
