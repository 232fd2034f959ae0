"""Build libhap.so (the HIP library behind include/hap.h) for gfx950 with hipcc.

    python -m paper_1403_7394_amd.build

compiles every HIP source under csrc/ into paper_1403_7394_amd/libhap.so.
Packed FP32 instructions are disabled (-packed-fp32-ops) for every HIP source.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libhap.so")
ARCH = "gfx950"

SOURCES = ["hap_api.hip", "sweep.hip", "select.hip", "misc.hip", "build.hip", "batch.hip", "warm.hip", "mlp.hip", "levelsim.hip", "fused.hip"]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def flags() -> list[str]:
    return [
        f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-fvisibility=hidden", "-Wall", "-Wno-unused-result",
        "-I", os.path.join(ROOT, "include"),
    ]


def build_library(verbose: bool = True, jobs: int = 8) -> str:
    """Compile each source to an object in parallel, then link libhap.so."""
    cc = hipcc()
    objdir = os.path.join(PKG, "_build")
    os.makedirs(objdir, exist_ok=True)
    procs = []
    objs = []
    base = [f for f in flags() if f != "-shared"]
    for src in SOURCES:
        obj = os.path.join(objdir, src.replace(".hip", ".o"))
        objs.append(obj)
        cmd = [cc, *base, "-c", os.path.join(CSRC, src), "-o", obj]
        procs.append((src, cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)))
        while sum(p.poll() is None for _, _, p in procs) >= jobs:
            procs[0][2].wait()
    failed = []
    for src, cmd, p in procs:
        out, _ = p.communicate()
        if verbose and out.strip():
            print(out, file=sys.stderr)
        if p.returncode != 0:
            failed.append((src, " ".join(cmd)))
    if failed:
        raise RuntimeError("hipcc failed for: " + ", ".join(s for s, _ in failed))
    tmp = LIB + ".tmp"
    link = [cc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(link, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        print(r.stdout, file=sys.stderr)
        raise RuntimeError("link failed")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    build_library()
