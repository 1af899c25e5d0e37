"""Host-only library code under AddressSanitizer and UndefinedBehaviorSanitizer:
the chunk / zone plan (checked against brute force on random column pointers),
the matrix fingerprint and the tuning cache, built with g++ from the library's
own sources (tests/native/host_check.cpp), plus the server's scheduling policy
(tests/native/sched_check.cpp) under the same sanitizers."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1812_00904_amd", "csrc")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]


def _build_and_run(tmp_path, name, sources, args=(), expect="ok"):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path / name)
    subprocess.check_call([gxx, "-std=c++17", "-O1", "-g", "-Wall", "-Werror"] + SAN +
                          ["-I", os.path.join(ROOT, "include"), "-I", CSRC] + sources + ["-o", exe])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe] + list(args), capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stdout + r.stderr
    assert expect in r.stdout


def test_plan_fingerprint_and_cache_under_sanitizers(tmp_path):
    _build_and_run(tmp_path, "host_check",
                   [os.path.join(ROOT, "tests", "native", "host_check.cpp"), os.path.join(CSRC, "spw_plan.cpp"),
                    os.path.join(CSRC, "spw_tune.cpp")], [str(tmp_path / "cache.txt")], "host ok")


def test_scheduler_under_sanitizers(tmp_path):
    _build_and_run(tmp_path, "sched_check", [os.path.join(ROOT, "tests", "native", "sched_check.cpp")],
                   expect="sched ok")
