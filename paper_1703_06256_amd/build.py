"""Build libhog.so (gfx950) in-tree with hipcc.

    python -m paper_1703_06256_amd.build

Compiles csrc/hog_kernels.hip for gfx950 and csrc/hog_api.cpp and
csrc/hog_server.cpp for the host, and links them into
paper_1703_06256_amd/libhog.so. Packed-FP32 instructions
are disabled for the device code.
"""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libhog.so")
BUILD_DIR = os.path.join(PKG, "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-I" + INCLUDE, "-I" + CSRC]
DEVICE = ["--offload-arch=" + ARCH, "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout)
        raise RuntimeError("build step failed: " + " ".join(cmd))
    return r.stdout


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD_DIR, exist_ok=True)
    k_obj = os.path.join(BUILD_DIR, "hog_kernels.o")
    a_obj = os.path.join(BUILD_DIR, "hog_api.o")
    s_obj = os.path.join(BUILD_DIR, "hog_server.o")
    steps = [
        [HIPCC, *COMMON, *DEVICE, "-c", os.path.join(CSRC, "hog_kernels.hip"), "-o", k_obj],
        [HIPCC, *COMMON, *DEVICE, "-x", "hip", "-c", os.path.join(CSRC, "hog_api.cpp"), "-o", a_obj],
        [HIPCC, *COMMON, *DEVICE, "-x", "hip", "-c", os.path.join(CSRC, "hog_server.cpp"), "-o", s_obj],
    ]
    for cmd in steps:
        out = _run(cmd)
        if verbose and out:
            print(out)
    tmp = LIB + ".tmp"
    _run([HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-pthread", "-o", tmp, k_obj, a_obj, s_obj])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
