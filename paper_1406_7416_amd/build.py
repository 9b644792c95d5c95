"""Build step: compiles the HIP library for gfx950 and the oracle's C library.

    python -m paper_1406_7416_amd.build
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# -ffp-contract=on: multiply-adds are fused only within one source expression, so a kernel
# body computes bitwise the same wherever it is inlined (per-problem and batched launches).
HIP_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared", "-ffp-contract=on",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"), "-Wall", "-Wno-unused-function",
]


def _run(cmd):
    print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)


def build_hip(jobs: int = 0) -> str:
    """Compiles every csrc/*.hip translation unit to an object (in parallel: the kernel
    instantiations are spread over several units) and links libadg.so."""
    from concurrent.futures import ThreadPoolExecutor
    srcs = sorted(glob.glob(os.path.join(PKG, "csrc", "*.hip")) + glob.glob(os.path.join(PKG, "csrc", "*.cpp")))
    if not srcs:
        return ""
    objdir = os.path.join(PKG, "_build")
    os.makedirs(objdir, exist_ok=True)
    cflags = [f for f in HIP_FLAGS if f != "-shared"]
    objs = [os.path.join(objdir, os.path.basename(src) + ".o") for src in srcs]
    jobs = jobs or min(len(srcs), max(1, min(16, os.cpu_count() or 1)))
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        list(ex.map(lambda so: _run([HIPCC, *cflags, "-c", so[0], "-o", so[1]]), zip(srcs, objs)))
    out = os.path.join(PKG, "libadg.so")
    tmp = out + ".tmp"
    _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp])
    os.replace(tmp, out)
    return out


def build_oracle() -> str:
    src = os.path.join(ROOT, "oracle", "adg_oracle.c")
    out = os.path.join(ROOT, "oracle", "liboracle.so")
    tmp = out + ".tmp"
    _run(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99", "-D_GNU_SOURCE", src, "-o", tmp, "-lm"])
    os.replace(tmp, out)
    return out


def build_all():
    build_oracle()
    build_hip()


if __name__ == "__main__":
    build_all()
    sys.exit(0)
