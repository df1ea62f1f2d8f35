"""The host planner and the pool allocator of libbcts (csrc/plan.cpp), built
on its own with g++ and the address and undefined-behaviour sanitizers, and
run against invariants of the plan (levels, eval segments, sibling groups,
chunks, the arena layout, per-request bytes), of the first-fit pool, and the
Eq. 6 / probit values (tests/host/plan_check.cpp)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="no host C++ compiler")
def test_planner_under_sanitizers(tmp_path):
    exe = str(tmp_path / "plan_check")
    src = [os.path.join(ROOT, "tests", "host", "plan_check.cpp"),
           os.path.join(ROOT, "paper_2107_01715_amd", "csrc", "plan.cpp")]
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-Wall", "-Wextra", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", *src, "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    env.pop("LD_PRELOAD", None)
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
