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

HIP_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"), "-Wall", "-Wno-unused-function",
]


def _run(cmd):
    print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)


def build_hip() -> str:
    srcs = sorted(glob.glob(os.path.join(PKG, "csrc", "*.hip")) + glob.glob(os.path.join(PKG, "csrc", "*.cpp")))
    if not srcs:
        return ""
    out = os.path.join(PKG, "libadg.so")
    tmp = out + ".tmp"
    _run([HIPCC, *HIP_FLAGS, *srcs, "-o", tmp])
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
