"""The serving loop's host core (csrc/serve_core.{h,cpp}: sessions, FIFO
admission by arena bytes and slots, tickets, cancellation, the failed state,
statistics, the worker loop) on the CPU with a fake executor, built with g++
under the address + undefined-behaviour sanitizers and under the thread
sanitizer (host code only: no HIP source is compiled here).  The checks are
in tests/serve_core_test.cpp."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2012_07145_amd", "csrc")


@pytest.mark.parametrize("sanitizer", ["address,undefined", "thread"])
def test_serve_core_under_sanitizer(tmp_path, sanitizer):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path / "serve_core_test")
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
           "-fsanitize=" + sanitizer, "-Wall", "-Wextra", "-Werror", "-pthread",
           "-I", os.path.join(ROOT, "include"), "-I", CSRC,
           os.path.join(ROOT, "tests", "serve_core_test.cpp"), os.path.join(CSRC, "serve_core.cpp"),
           "-o", exe]
    b = subprocess.run(cmd, capture_output=True, text=True)
    assert b.returncode == 0, b.stdout + b.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1",
               TSAN_OPTIONS="halt_on_error=1:second_deadlock_stack=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "all checks passed" in r.stdout
