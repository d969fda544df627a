"""Builds libibmpoisson.so (hipcc, gfx950) in-tree.

Every translation unit is compiled for gfx950 only with packed-FP32
instructions disabled; the classification, ghost-stencil and surface-load
and advection-diffusion units are compiled without FMA contraction so their
quantisation,
predicates, distance comparisons and interpolations round exactly as
written.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libibmpoisson.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

UNITS = {
    "capi.hip": [],
    "memory.hip": [],
    "classify.hip": ["-ffp-contract=off"],
    "stencils.hip": ["-ffp-contract=off"],
    "solver.hip": [],
    "server.hip": [],
    "forces.hip": ["-ffp-contract=off"],
    "ad.hip": ["-ffp-contract=off"],
    "stream.hip": [],
}

COMMON = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang",
          "-packed-fp32-ops", "-Wno-unused-command-line-argument", "-I", os.path.join(ROOT, "include"), "-I", CSRC]


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    procs = []
    objs = []
    for src, extra in UNITS.items():
        path = os.path.join(CSRC, src)
        if not os.path.exists(path):
            continue
        obj = os.path.join(BUILD, src.replace(".hip", ".o"))
        objs.append(obj)
        cmd = [HIPCC, *COMMON, *extra, "-c", path, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
    failed = []
    for src, p in procs:
        out, _ = p.communicate()
        txt = out.decode(errors="replace")
        txt = "\n".join(l for l in txt.splitlines() if "packed-fp32-ops" not in l and "not a recognized feature" not in l
                        and l.strip() != "1 warning generated.")
        if txt.strip() and (verbose or p.returncode):
            print(txt, file=sys.stderr)
        if p.returncode:
            failed.append(src)
    if failed:
        raise RuntimeError("hipcc failed for " + ", ".join(failed))
    tmp = LIB + ".tmp%d" % os.getpid()
    subprocess.check_call([HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp, *objs, "-lpthread"])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
