"""Build the serving stress driver (session_stress.cpp) against the library's host runtime
compiled with a sanitizer, on the CPU.

The host sources (runtime, session, replay harness) and the driver are compiled by ROCm's host
clang++ with -fsanitize=thread or -fsanitize=address (its runtimes intercept the timed
condition-variable waits of libstdc++, which GCC 11's ThreadSanitizer does not, and reports
false double locks for); the device sources come from the library's normal build
(paper_2412_13043_amd/_build, compiled by hipcc without any sanitizer).  Only the fake executor
runs, so no GPU is needed.  Usage: python build_sanitized.py thread|address OUTDIR
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
CSRC = os.path.join(ROOT, "paper_2412_13043_amd", "csrc")
BUILD = os.path.join(ROOT, "paper_2412_13043_amd", "_build")
HOST = ["frg_runtime.cpp", "frg_session.cpp", "frg_replay.cpp"]
CXX = "/opt/rocm/llvm/bin/clang++"
DEVICE_OBJS = ["frg_kernels.o", "frg_stepper.o", "frg_threshold.o", "frg_noalloc.o",
               "frg_flop_probe.o"]


def build(kind: str, out_dir: str) -> str:
    assert kind in ("thread", "address")
    os.makedirs(out_dir, exist_ok=True)
    flags = ["-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=" + kind,
             "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", "-I" + os.path.join(ROOT, "include")]
    objs = []
    for src in HOST + [os.path.join(HERE, "session_stress.cpp")]:
        path = src if os.path.isabs(src) else os.path.join(CSRC, src)
        obj = os.path.join(out_dir, os.path.basename(src).rsplit(".", 1)[0] + ".o")
        subprocess.check_call([CXX, "-c"] + flags + [path, "-o", obj])
        objs.append(obj)
    for o in DEVICE_OBJS:
        p = os.path.join(BUILD, o)
        if not os.path.exists(p):
            raise FileNotFoundError(f"{p} is missing: build the library first")
        objs.append(p)
    exe = os.path.join(out_dir, "session_stress_" + kind)
    subprocess.check_call([CXX, "-fsanitize=" + kind, "-o", exe] + objs +
                          ["-L/opt/rocm/lib", "-Wl,-rpath,/opt/rocm/lib", "-lamdhip64",
                           "-lpthread"])
    return exe


if __name__ == "__main__":
    print(build(sys.argv[1], sys.argv[2]))
