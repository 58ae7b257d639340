"""Builds libug.so (the HIP kernels + C ABI) in-tree for gfx950 with hipcc.

Usage: ``python -m paper_2505_05643_amd.build`` (or ``build()``).  Every call
recompiles; object files go to ``_build/`` next to this file.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
OBJDIR = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libug.so")

SOURCES = ["ug_api.hip", "ug_preprocess.hip", "ug_sort.hip", "ug_raster.hip", "ug_scatter.hip", "ug_densify.hip",
           "ug_train.hip", "ug_quality.hip", "ug_params.hip", "ug_probe.hip"]

ARCH = "gfx950"
HIPCC_FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # Packed FP32 (v_pk_*_f32) stays off: only scalar FP32 VALU forms are emitted.
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
    "-I", INCLUDE, "-I", CSRC,
]


def _hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm is required to build libug)")


def build(verbose: bool = False, jobs: int | None = None) -> str:
    hipcc = _hipcc()
    os.makedirs(OBJDIR, exist_ok=True)
    procs = []
    objs = []
    jobs = jobs or min(len(SOURCES), os.cpu_count() or 1, 8)
    pending = list(SOURCES)
    running = []
    while pending or running:
        while pending and len(running) < jobs:
            src = pending.pop(0)
            obj = os.path.join(OBJDIR, src.replace(".hip", ".o"))
            objs.append(obj)
            cmd = [hipcc, *HIPCC_FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
            if verbose:
                print(" ".join(cmd), flush=True)
            running.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        src, pr = running.pop(0)
        out, _ = pr.communicate()
        text = out.decode(errors="replace")
        # hipcc's host pass does not know the gfx950 feature name: harmless.
        lines = [l for l in text.splitlines() if "packed-fp32-ops" not in l and l.strip()]
        if pr.returncode != 0:
            raise RuntimeError(f"hipcc failed on {src}:\n{text}")
        if verbose and lines:
            print("\n".join(lines), flush=True)
        procs.append(src)
    tmp = LIB + ".tmp"
    cmd = [hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stdout.decode(errors="replace"))
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
