"""Scheduler of the served path (em_serve.cpp) on a fake device, on the CPU.

The serving loop is compiled against host stand-ins for the HIP calls and for
the pipeline stages (tests/serve_host), under ThreadSanitizer, and driven
through map_submit / map_poll: every job completes with the right outputs,
slots and the device-memory budget bound what is in flight, one slot admits
in submission order, oversized jobs and a full queue are refused at submit,
zero-timeout polls return at once, a failing job reports its own error and
leaves the others untouched, shutdown drains all jobs, and many contexts in a
row with random sizes run clean (no data race, no lock-order problem).
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CLANG = "/opt/rocm/llvm/bin/clang++"


def test_serving_scheduler_on_fake_device(tmp_path):
    cxx = CLANG if os.path.exists(CLANG) else shutil.which("clang++")
    if cxx is None:
        pytest.skip("clang++ with ThreadSanitizer not available")
    exe = str(tmp_path / "serve_host")
    src = [os.path.join(ROOT, "paper_2404_17084_amd", "csrc", "em_serve.cpp"),
           os.path.join(ROOT, "tests", "serve_host", "fake_device.cpp"),
           os.path.join(ROOT, "tests", "serve_host", "driver.cpp")]
    inc = ["-I" + os.path.join(ROOT, "tests", "serve_host"),
           "-I" + os.path.join(ROOT, "paper_2404_17084_amd", "csrc"), "-I" + os.path.join(ROOT, "include")]
    subprocess.check_call([cxx, "-std=c++17", "-O1", "-g", "-fsanitize=thread"] + inc + src + ["-o", exe, "-lpthread"])
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1 exitcode=66")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr[-4000:]
    assert "all scenarios passed" in r.stdout
