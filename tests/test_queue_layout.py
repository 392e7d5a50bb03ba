"""CPU test of the stage-batched plans' launch layout (queue_layout.h): random mixes of
cells over graph branches and kernel variants; every (cell, step) lands in exactly one
launch of its step, branch and variant; segments are end to end on multiples of 8
workgroups; the cells' order alternates by step; the binary-search lookup the kernels
use maps every workgroup back to its cell (and its XCD to the one of the cell's own
launch), and the rounding workgroups to none; mismatched pipelines and oversized
launches are refused.  The C++ test program is built with g++."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "queue_layout_test.cpp")
INC = os.path.join(ROOT, "paper_2607_05920_amd", "csrc")


def test_queue_layout(tmp_path):
    if not shutil.which("g++"):
        pytest.skip("g++ not available")
    exe = tmp_path / "queue_layout_test"
    r = subprocess.run(["g++", "-std=c++17", "-O2", "-I", INC, SRC, "-o", str(exe)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and "ALL PASSED" in r.stdout, r.stdout + r.stderr
