"""Builds libdecmg.so in-tree with hipcc for gfx950.

Run as ``python -m paper_2508_12501_amd.build``.  Objects go to ``_build/`` at the
repository root; the shared library lands next to this file.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libdecmg.so")
BUILD = os.path.join(ROOT, "_build")

ARCH = "gfx950"
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
COMMON = ["-O3", "-fPIC", "-std=c++17", f"-I{os.path.join(ROOT, 'include')}", f"-I{CSRC}"]
# no packed FP32 instructions in device code
DEVICE = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
# host sources whose arithmetic must follow plain IEEE order (mesh geometry, row sums)
STRICT_HOST = {"mesh.cpp", "hierarchy.cpp"}

SOURCES = ["mesh.cpp", "geomap.cpp", "hierarchy.cpp", "solver.cpp", "capi.cpp", "porous.cpp", "porous_rk.cpp", "batch.cpp", "kernels.hip", "porous.hip", "batch.hip"]


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"build step failed: {' '.join(cmd[:3])} ... ({r.returncode})")


def _jobs() -> int:
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        n = os.cpu_count() or 1
    return max(1, min(n, 16, int(os.environ.get("MAX_JOBS", n))))


def build(verbose: bool = False) -> str:
    cc = hipcc()
    os.makedirs(BUILD, exist_ok=True)
    cmds, objs = [], []
    for src in SOURCES:
        path = os.path.join(CSRC, src)
        obj = os.path.join(BUILD, src + ".o")
        cmd = [cc, f"--offload-arch={ARCH}", *COMMON]
        if src.endswith(".hip"):
            cmd += DEVICE
        else:
            cmd += ["-x", "c++", "-D__HIP_PLATFORM_AMD__", f"-I{ROCM}/include"]
        if src in STRICT_HOST:
            cmd += ["-ffp-contract=off"]
        cmd += ["-c", path, "-o", obj]
        cmds.append(cmd)
        objs.append(obj)
    # the device sources take longest: start them first
    order = sorted(range(len(cmds)), key=lambda i: not SOURCES[i].endswith(".hip"))
    with ThreadPoolExecutor(max_workers=_jobs()) as ex:
        for f in [ex.submit(_run, cmds[i], verbose) for i in order]:
            f.result()
    tmp = OUT + ".tmp"
    _run([cc, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp], verbose)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
