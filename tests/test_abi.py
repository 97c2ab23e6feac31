"""C-ABI checks that need no GPU: the library loads, exports every function include/frg.h
declares, the ctypes structs match the C layouts, and argument errors are reported without any
device work."""
import ctypes
import os
import re
import subprocess

import pytest

from paper_2412_13043_amd import frg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "frg.h")


def _declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:frg_status|const char \*)\s*(frg_\w+)\s*\(", text,
                                 re.M)))


def test_header_declares_the_abi():
    names = _declared_functions()
    assert "frg_integrate_batch" in names and "frg_flow_rhs" in names
    assert "frg_session_submit" in names and "frg_integrate_multi" in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(frg.LIB_PATH)
    for name in _declared_functions():
        assert hasattr(lib, name), name
    assert sorted(frg.EXPORTED) == _declared_functions()
    nm = subprocess.run(["nm", "-D", "--defined-only", frg.LIB_PATH], capture_output=True,
                        text=True, check=True).stdout
    exported = set(re.findall(r"\sT\s(frg_\w+)$", nm, re.M))
    assert set(_declared_functions()) <= exported


def test_struct_layouts_match_c(tmp_path):
    src = tmp_path / "sz.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "frg.h"\n'
                   'int main(void){printf("%zu %zu %zu %zu %zu %zu %zu\\n",'
                   'sizeof(frg_integral_desc), sizeof(frg_batch), sizeof(frg_flow_state),'
                   'sizeof(frg_session_config), sizeof(frg_stats),'
                   'offsetof(frg_batch, out), offsetof(frg_flow_state, coef));return 0;}\n')
    exe = tmp_path / "sz"
    subprocess.run(["gcc", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
                    "-I" + os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True,
                                          check=True).stdout.split()]
    want = [ctypes.sizeof(frg.frg_integral_desc), ctypes.sizeof(frg.frg_batch),
            ctypes.sizeof(frg.frg_flow_state), ctypes.sizeof(frg.frg_session_config),
            ctypes.sizeof(frg.frg_stats), frg.frg_batch.out.offset, frg.frg_flow_state.coef.offset]
    assert got == want


def test_null_context_is_rejected_without_device_work():
    desc = frg.make_desc(frg.FRG_FAMILY_LPA, 32, 6.0)
    b = frg.frg_batch()
    st = frg.raw_status("frg_integrate_batch", None, ctypes.byref(desc), ctypes.byref(b), None)
    assert st == frg.FRG_E_INVAL
    assert "context" in frg.frg_last_error()
    st = frg.raw_status("frg_flow_rhs", None, ctypes.byref(desc), None, None, None)
    assert st == frg.FRG_E_INVAL
    st = frg.raw_status("frg_integrate_multi", None, 1, None, None, None)
    assert st == frg.FRG_E_INVAL
    st = frg.raw_status("frg_integrate_batch_noalloc", None, ctypes.byref(desc),
                        ctypes.byref(b), None)
    assert st == frg.FRG_E_INVAL


def test_context_create_rejects_bad_arguments():
    st = frg.raw_status("frg_context_create", 0, 0, None)
    assert st == frg.FRG_E_INVAL
    h = ctypes.c_void_p()
    st = frg.raw_status("frg_context_create", -1, 0, ctypes.byref(h))
    assert st in (frg.FRG_E_INVAL, frg.FRG_E_DEVICE)
    assert frg.frg_last_error() != ""


def test_destroy_null_is_noop():
    assert frg.raw_status("frg_context_destroy", None) == frg.FRG_OK


def test_binding_loads_a_single_hip_runtime():
    # the binding imports torch first, so libfrg.so binds to torch's HIP runtime
    import subprocess
    import sys

    code = ("from paper_2412_13043_amd import frg\n"
            "m = open('/proc/self/maps').read().splitlines()\n"
            "print(len({l.split()[-1] for l in m if 'libamdhip64' in l}))\n")
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True,
                         cwd=ROOT, check=True).stdout.split()
    assert out[-1] == "1"


def test_library_exports_every_testing_symbol():
    text = open(os.path.join(ROOT, "include", "frg_testing.h")).read()
    names = sorted(set(re.findall(r"^\s*(?:frg_status|void)\s*(frg_\w+)\s*\(", text, re.M)))
    assert "frg_serving_replay" in names and "frg_session_open_fake" in names
    assert sorted(frg.TESTING_EXPORTED) == names
    lib = ctypes.CDLL(frg.LIB_PATH)
    for name in names:
        assert hasattr(lib, name), name
