"""The host plan (ring checks, lifts, plans of both transforms, decoding
matrices and their cache, the light Cauchy search, error paths) built with
g++ under AddressSanitizer and UndefinedBehaviorSanitizer and driven by
tests/native/plan_check.cpp.  CPU only: the plan code is plain C++ and
compiles without hipcc."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not installed")
def test_host_plan_under_sanitizers(tmp_path):
    exe = tmp_path / "plan_check"
    build = ["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined",
             "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-pthread",
             "-I" + os.path.join(ROOT, "include"),
             os.path.join(ROOT, "paper_1709_00178_amd", "csrc", "plan.cpp"),
             os.path.join(ROOT, "tests", "native", "plan_check.cpp"), "-o", str(exe)]
    r = subprocess.run(build, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0 and r.stdout.strip() == "ok", (r.stdout + r.stderr)[-4000:]
