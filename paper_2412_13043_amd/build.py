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
    ("frg_stepper.hip", True),
    ("frg_threshold.hip", True),
    ("frg_noalloc.hip", True),
    ("frg_flop_probe.hip", True),
    ("frg_runtime.cpp", False),
    ("frg_session.cpp", False),
    ("frg_replay.cpp", False),
]


def _run(cmd):
    print("+", " ".join(cmd), flush=True)
    subprocess.check_call(cmd)


def build(verbose: bool = True, out: str = LIB, defines=(), csrc: str = CSRC) -> str:
    """Compile and link libfrg.so; `defines` are extra -D tuning macros for the device code;
    `csrc` another directory with the same sources (a modified copy, for measurements)."""
    build_dir = BUILD if out == LIB else out + ".build"
    os.makedirs(build_dir, exist_ok=True)
    objs = []
    for src, is_device in SOURCES:
        obj = os.path.join(build_dir, src.rsplit(".", 1)[0] + ".o")
        cmd = ["hipcc", "-c"] + COMMON
        if is_device:
            cmd += DEVICE + ["-D" + d for d in defines]
        else:
            cmd += ["-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", "-x", "c++"]
        cmd += [os.path.join(csrc, src), "-o", obj]
        _run(cmd)
        objs.append(obj)
    tmp = out + ".tmp"
    _run(["hipcc", "-shared", "-o", tmp] + objs + ["--offload-arch=" + ARCH, "-lpthread"])
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    # python build.py [OUT.so [MACRO=VALUE ...]]
    if len(sys.argv) > 1:
        build(out=os.path.abspath(sys.argv[1]), defines=sys.argv[2:])
    else:
        build()
    sys.exit(0)
