"""The serving loop's host code under ThreadSanitizer and AddressSanitizer (CPU only).

tests/sanitize/build_sanitized.py compiles the host runtime, the session and the replay harness
with a sanitizer and links tests/sanitize/session_stress.cpp against them (device objects from
the normal build); the driver runs fake sessions only: many client threads, cancellation, split
requests, admission under a small budget, injected launch failures, the watchdog, the replay
harness, close while busy and argument errors.  Any sanitizer report fails the test."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, os.path.join(ROOT, "tests", "sanitize"))

CXX = "/opt/rocm/llvm/bin/clang++"


@pytest.mark.skipif(not os.path.exists(CXX), reason="ROCm host clang++ not found")
@pytest.mark.parametrize("kind", ["thread", "address"])
def test_session_stress_is_sanitizer_clean(kind, tmp_path):
    import build_sanitized

    exe = build_sanitized.build(kind, str(tmp_path))
    env = dict(os.environ)
    env["TSAN_OPTIONS"] = "halt_on_error=1 second_deadlock_stack=1"
    env["ASAN_OPTIONS"] = "detect_leaks=1 halt_on_error=1"
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env, cwd=tmp_path)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "ThreadSanitizer" not in out and "AddressSanitizer" not in out, out[-4000:]
    assert "LeakSanitizer" not in out, out[-4000:]
    assert "session stress: ok" in out
