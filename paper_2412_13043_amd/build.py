"""Build the HIP library libfrg.so for gfx950 in-tree (hipcc; no JIT, no torch extension)."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libfrg.so")
ARCH = os.environ.get("FRG_OFFLOAD_ARCH", "gfx950")

COMMON = ["-std=c++17", "-O3", "-fPIC", "-Wall", "-Wno-unused-function", "-ffp-contract=off",
          "-I" + os.path.join(HERE, "..", "include")]
# device code: gfx950 only; packed-FP32 instruction forms are disabled
DEVICE = ["--offload-arch=" + ARCH, "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-munsafe-fp-atomics"]

SOURCES = [
    ("frg_kernels.hip", True),
    ("frg_runtime.cpp", False),
    ("frg_session.cpp", False),
]


def _run(cmd):
    print("+", " ".join(cmd), flush=True)
    subprocess.check_call(cmd)


def build(verbose: bool = True) -> str:
    os.makedirs(BUILD, exist_ok=True)
    objs = []
    for src, is_device in SOURCES:
        obj = os.path.join(BUILD, src.rsplit(".", 1)[0] + ".o")
        cmd = ["hipcc", "-c"] + COMMON
        if is_device:
            cmd += DEVICE
        else:
            cmd += ["-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", "-x", "c++"]
        cmd += [os.path.join(CSRC, src), "-o", obj]
        _run(cmd)
        objs.append(obj)
    tmp = LIB + ".tmp"
    _run(["hipcc", "-shared", "-o", tmp] + objs + ["--offload-arch=" + ARCH, "-lpthread"])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build()
    sys.exit(0)
