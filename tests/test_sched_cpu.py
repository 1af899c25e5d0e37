"""The server's scheduling policy (pure host code) built with g++ and checked
on hand-made queues: merging by matrix / operation / vector type in arrival
order, the column cap, stream affinity of a matrix with work in flight, the
per-stream depth limit and the least-busy stream choice."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_sched_policy(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path / "sched_check")
    subprocess.check_call([gxx, "-std=c++17", "-O1", "-Wall", "-Werror",
                           "-I", os.path.join(ROOT, "paper_1812_00904_amd", "csrc"),
                           os.path.join(ROOT, "tests", "native", "sched_check.cpp"), "-o", exe])
    r = subprocess.run([exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "sched ok" in r.stdout
