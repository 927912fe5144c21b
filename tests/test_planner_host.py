"""The encode planner (host code: part boundaries, attention work items,
descriptors, capacity buckets, workspace layout) built on its own with
AddressSanitizer and UndefinedBehaviorSanitizer and run over seeded random
batches; tests/planner_check.cpp holds the checks."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2505_00690_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="no host C++ compiler")
def test_planner_under_sanitizers(tmp_path):
    exe = str(tmp_path / "planner_check")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-Wall", "-Werror",
           "-I", CSRC, os.path.join(ROOT, "tests", "planner_check.cpp"),
           os.path.join(CSRC, "plan.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    env.pop("LD_PRELOAD", None)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.startswith("ok "), r.stdout
    counts = dict(kv.split("=") for kv in r.stdout.split()[1:])
    assert int(counts["plans"]) == 1500
    assert int(counts["two_part"]) > 50 and int(counts["same_bucket_pairs"]) > 50
    assert int(counts["refused"]) == 9
