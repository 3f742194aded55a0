"""Builds libcloth.so (the HIP library behind include/cloth.h) for gfx950.

Usage: python paper_2403_19272_amd/build.py   (or build() from this module; importing
the package itself needs the built library).
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libcloth.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

COMMON = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-I", os.path.join(HERE, "..", "include")]
SOURCES = [
    # (source, extra flags)
    ("host_build.cpp", []),
    ("api.cpp", ["-fopenmp"]),
    ("serve.cpp", []),
    ("tune.cpp", []),
    ("pd_kernels.hip", []),
    ("eig.hip", []),
    # FP64 geometric predicates: keep the written operation order
    ("contact_kernels.hip", ["-ffp-contract=off"]),
]


def build(verbose: bool = False) -> str:
    os.makedirs(OBJ, exist_ok=True)
    objs = []
    for src, extra in SOURCES:
        out = os.path.join(OBJ, os.path.splitext(src)[0] + ".o")
        lang = ["-x", "hip"] if src.endswith(".hip") else []
        cmd = [HIPCC, *COMMON, *extra, *lang, "-c", os.path.join(CSRC, src), "-o", out]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        objs.append(out)
    tmp = LIB + ".tmp"
    # -z defs: an unresolved symbol fails the link instead of the first load
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fopenmp", "-pthread", "-Wl,-z,defs", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
