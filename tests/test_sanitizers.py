"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer.

* The oracle's C code: a small C driver (tests/sanitize/oracle_driver.c) calls every entry point on
  a tiny odd-sized geometry, with view subsets, the step-rule options and the filtered
  backprojection.
* The library's host code: the whole library built with the sanitizers on its host side only
  (hipcc -Xarch_host), driven by tests/sanitize/library_driver.cpp through the ray tables and the
  gather's window check, the batched kernels' work tables and the argument checks every entry point
  runs before it touches the device (no GPU is used).

Any out-of-bounds access, use after free or undefined operation aborts the run.  (The GPU path has
no atomics; its determinism tests stand in for a race detector.)"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_sanitizers(tmp_path):
    exe = tmp_path / "oracle_driver"
    cmd = ["gcc", "-O1", "-g", "-std=c11", "-fopenmp", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", os.path.join(ROOT, "tests", "sanitize", "oracle_driver.c"),
           os.path.join(ROOT, "oracle", "oracle.c"), "-lm", "-o", str(exe)]
    subprocess.run(cmd, check=True, capture_output=True)
    env = dict(os.environ, OMP_NUM_THREADS="2",
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=120)
    assert r.returncode == 0, r.stderr[-2000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
    assert r.stdout.startswith("rc 0")


HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.mark.timeout(600)
@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")
def test_library_host_code_under_sanitizers(tmp_path):
    csrc = os.path.join(ROOT, "paper_1903_10088_amd", "csrc")
    srcs = [os.path.join(csrc, f) for f in ("kernels.hip", "bp.hip", "api.hip", "batch.hip", "cnn.hip", "fbp.hip",
                                             "rebin.hip")]
    exe = tmp_path / "library_driver"
    cmd = [HIPCC, "-O1", "-g", "-std=c++17", "--offload-arch=gfx950",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer",
           "-I", os.path.join(ROOT, "include"), "-I", csrc, *srcs,
           os.path.join(ROOT, "tests", "sanitize", "library_driver.cpp"), "-o", str(exe)]
    b = subprocess.run(cmd, capture_output=True, text=True)
    assert b.returncode == 0, b.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-2000:])
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
    assert "failures 0" in r.stdout
