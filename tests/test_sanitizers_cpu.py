"""CPU tests: the host planner and the oracle built with AddressSanitizer and
UndefinedBehaviorSanitizer (host code only; no GPU code is built here) and
run on small meshes of every kind (tests/sanitize/).  Any out-of-bounds
access, leak or undefined behaviour fails the run."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = os.path.join(ROOT, "tests", "sanitize")
FLAGS = ["-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer"]


def _run(cmd, tmp_path, name):
    exe = str(tmp_path / name)
    r = subprocess.run(cmd + ["-o", exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    env.pop("LD_PRELOAD", None)
    p = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert p.returncode == 0, (p.stdout[-2000:], p.stderr[-6000:])
    return p.stdout


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_planner_under_asan_ubsan(tmp_path):
    csrc = os.path.join(ROOT, "paper_2107_11541_amd", "csrc")
    cmd = ["g++", "-std=c++17", "-pthread", *FLAGS, "-I", os.path.join(ROOT, "include"),
           os.path.join(SAN, "plan_check.cpp"), os.path.join(csrc, "plan.cpp"), os.path.join(csrc, "rowplan.cpp"),
           os.path.join(csrc, "symmap.cpp")]
    out = _run(cmd, tmp_path, "plan_check")
    assert "0 failed checks" in out


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_asan_ubsan(tmp_path):
    cmd = ["gcc", "-std=gnu99", "-ffp-contract=off", *FLAGS, os.path.join(SAN, "oracle_check.c"), "-lm"]
    out = _run(cmd, tmp_path, "oracle_check")
    assert "0 failures" in out
