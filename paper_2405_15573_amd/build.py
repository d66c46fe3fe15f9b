"""Compile the native parts of the package in-tree.

* ``libuhm_builder.so``: host operator construction (g++ -O3 -fopenmp).
* ``libuhm.so``: the HIP kernels and the C-ABI of include/uhm.h, for gfx950 only.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

HIP_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-munsafe-fp-atomics", "-Wall",
]


def _run(cmd):
    print("+", " ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)


def build_builder() -> str:
    out = os.path.join(HERE, "libuhm_builder.so")
    _run(["g++", "-O3", "-march=x86-64-v2", "-fopenmp", "-fPIC", "-shared", "-std=c++17", "-Wall",
          os.path.join(CSRC, "builder_native.cpp"), "-o", out])
    return out


def build_hip() -> str:
    out = os.path.join(HERE, "libuhm.so")
    srcs = [os.path.join(CSRC, f) for f in sorted(os.listdir(CSRC)) if f.endswith(".hip")]
    if not srcs:
        return ""
    _run([HIPCC, *HIP_FLAGS, "-I", os.path.join(ROOT, "include"), *srcs, "-o", out])
    return out


def build_all() -> None:
    build_builder()
    build_hip()


if __name__ == "__main__":
    what = sys.argv[1:] or ["all"]
    for w in what:
        {"builder": build_builder, "hip": build_hip, "all": build_all}[w]()
