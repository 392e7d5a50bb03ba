"""CPU tests of the request loop's scheduler core against a mock executor (a fake
device whose batches complete after a set delay, with injectable errors): batching
by cell, oldest-first service, scheduled arrivals, admission by the memory budget
(budget 0, oversized requests, batches cut to fit, waiting for memory), injected
launch and device errors, cancellation, and concurrent submitters.  The C++ test
program is built with g++ and run twice: plainly, and under ThreadSanitizer."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "srv_core_test.cpp")
INC = os.path.join(ROOT, "paper_2607_05920_amd", "csrc")


def _build_and_run(tmp_path, extra):
    if not shutil.which("g++"):
        pytest.skip("g++ not available")
    exe = tmp_path / "srv_core_test"
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-pthread", "-I", INC, SRC, "-o", str(exe)] + extra
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1 second_deadlock_stack=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120, env=env)
    assert r.returncode == 0 and "ALL PASSED" in r.stdout, r.stdout + r.stderr
    return r.stdout


def test_scheduler_core_with_mock_executor(tmp_path):
    out = _build_and_run(tmp_path, [])
    assert "concurrent_submitters" in out


def test_scheduler_core_under_thread_sanitizer(tmp_path):
    probe = subprocess.run(["g++", "-fsanitize=thread", "-x", "c++", "-", "-o", str(tmp_path / "p")],
                           input="int main(){return 0;}", capture_output=True, text=True)
    if probe.returncode != 0:
        pytest.skip("ThreadSanitizer not available")
    # GCC 11's TSan runtime does not intercept the steady-clock condition wait
    _build_and_run(tmp_path, ["-fsanitize=thread", "-DFHE_SRV_SYSTEM_CLOCK_WAIT"])
