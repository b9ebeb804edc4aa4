"""Host code built with g++ under AddressSanitizer and
UndefinedBehaviorSanitizer: the plan (ring checks, lifts, plans of both
transforms, decoding matrices and their cache, the light Cauchy search,
error paths; driven by tests/native/plan_check.cpp) and the batch builder
(driven by tests/native/batch_check.cpp).  CPU only: neither needs hipcc or a
GPU."""
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


ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


@pytest.mark.skipif(shutil.which("g++") is None or not os.path.exists(os.path.join(ROCM, "lib", "libamdhip64.so")),
                    reason="g++ or the HIP runtime library not installed")
def test_batch_builder_under_sanitizers(tmp_path):
    """pyrit_batch_describe on seeded random mixed batches (every kernel ring,
    both transforms, encodes and decodes, ragged and padded slices) with every
    executor, driven by tests/native/batch_check.cpp: passes and bytes moved
    against their closed forms, XCD ranges adding up, grid sizes; the
    builder's host code under AddressSanitizer and UndefinedBehaviorSanitizer.
    The HIP runtime is linked for its symbols only: nothing calls the device."""
    exe = tmp_path / "batch_check"
    csrc = os.path.join(ROOT, "paper_1709_00178_amd", "csrc")
    build = ["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined",
             "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-pthread",
             "-D__HIP_PLATFORM_AMD__", f"-I{ROCM}/include", "-I" + os.path.join(ROOT, "include"),
             os.path.join(csrc, "batch_host.cpp"), os.path.join(csrc, "plan.cpp"),
             os.path.join(ROOT, "tests", "native", "batch_check.cpp"),
             f"-L{ROCM}/lib", "-lamdhip64", f"-Wl,-rpath,{ROCM}/lib", "-o", str(exe)]
    r = subprocess.run(build, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0 and r.stdout.strip() == "ok", (r.stdout + r.stderr)[-4000:]


@pytest.mark.skipif(shutil.which("g++") is None or not os.path.exists(os.path.join(ROCM, "lib", "libamdhip64.so")),
                    reason="g++ or the HIP runtime library not installed")
def test_load_store_addresses_stay_in_blocks(tmp_path):
    """Every load and store address of the plain kernel (4-, 8- and 16-byte
    lanes) and of the batch executors (grid, split-K pairs, XCD order, queue,
    static) on seeded batches with ragged and padded slices lies inside its
    block, under either reading of the raw-buffer range check (with or
    without soffset); driven by tests/native/address_check.cpp over the real
    batch builder, which also shows that the old rule (lanes past the end of
    a slice loading at their own column) reads past the end of a block."""
    exe = tmp_path / "address_check"
    csrc = os.path.join(ROOT, "paper_1709_00178_amd", "csrc")
    build = ["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined",
             "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-pthread",
             "-D__HIP_PLATFORM_AMD__", f"-I{ROCM}/include", "-I" + os.path.join(ROOT, "include"),
             os.path.join(csrc, "batch_host.cpp"), os.path.join(csrc, "plan.cpp"),
             os.path.join(ROOT, "tests", "native", "address_check.cpp"),
             f"-L{ROCM}/lib", "-lamdhip64", f"-Wl,-rpath,{ROCM}/lib", "-o", str(exe)]
    r = subprocess.run(build, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0 and r.stdout.strip() == "ok", (r.stdout + r.stderr)[-4000:]


@pytest.mark.skipif(shutil.which("g++") is None or not os.path.exists(os.path.join(ROCM, "lib", "libamdhip64.so")),
                    reason="g++ or the HIP runtime library not installed")
def test_failed_host_allocations_return_enomem(tmp_path):
    """No C++ exception crosses the C ABI: with the global operator new made
    to fail at its 1st, 2nd, ... allocation, pyrit_lift, pyrit_plan_create_ex
    (both transforms), pyrit_decode_matrix, pyrit_cauchy_light and
    pyrit_batch_describe (every executor) return PYRIT_ENOMEM until the call
    gets through, then the undisturbed result; nothing leaks (AddressSanitizer
    leak check).  Driven by tests/native/alloc_fail_check.cpp."""
    exe = tmp_path / "alloc_fail_check"
    csrc = os.path.join(ROOT, "paper_1709_00178_amd", "csrc")
    build = ["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined",
             "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-pthread",
             "-D__HIP_PLATFORM_AMD__", f"-I{ROCM}/include", "-I" + os.path.join(ROOT, "include"),
             os.path.join(csrc, "batch_host.cpp"), os.path.join(csrc, "plan.cpp"),
             os.path.join(ROOT, "tests", "native", "alloc_fail_check.cpp"),
             f"-L{ROCM}/lib", "-lamdhip64", f"-Wl,-rpath,{ROCM}/lib", "-o", str(exe)]
    r = subprocess.run(build, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0 and r.stdout.strip() == "ok", (r.stdout + r.stderr)[-4000:]
