"""AddressSanitizer and UndefinedBehaviorSanitizer builds of host code (no GPU code is
instrumented; none of this needs a GPU).

* The CPU oracle: tests/sanitize/oracle_driver.c calls every oracle entry point on a small
  polar jet grid and a skewed periodic box, and the invalid-parameter paths. It is compiled
  with oracle/oracle.c by gcc with -fsanitize=address,undefined (no OpenMP, so the
  sanitizers see one thread).
* The library's host code: a build of the HIP sources for gfx950 with the sanitizers passed to
  the host compilation only (-Xarch_host), driven by tests/sanitize/host_driver.c
  through every C-ABI path that returns before a device call (parameter validation,
  including the largest-grid limit, null handles and arguments, the tuning table).

Each must run clean: exit status 0 and no sanitizer report.
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_runs_clean_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_driver")
    cmd = ["gcc", "-O1", "-g", "-std=c99", "-D_DEFAULT_SOURCE", "-ffp-contract=off",
           "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", "-Wno-unknown-pragmas",
           os.path.join(HERE, "sanitize", "oracle_driver.c"),
           os.path.join(ROOT, "oracle", "oracle.c"), "-o", exe, "-lm"]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    res = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert res.returncode == 0, res.stdout + res.stderr
    assert "oracle driver ok" in res.stdout
    assert "runtime error" not in res.stderr and "AddressSanitizer" not in res.stderr, res.stderr


HIPCC = "/opt/rocm/bin/hipcc"
CLANG = "/opt/rocm/llvm/bin/clang"
CSRC = os.path.join(ROOT, "paper_2212_12365_amd", "csrc")
SOURCES = ["lesmi.hip", "les_stage.hip", "les_batch.hip", "les_mlp.hip", "les_fwh.hip"]


@pytest.mark.skipif(not (os.path.exists(HIPCC) and os.path.exists(CLANG)),
                    reason="ROCm compilers not available")
def test_library_host_code_runs_clean_under_asan_and_ubsan(tmp_path):
    lib = str(tmp_path / "liblesmi_hostsan.so")
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=undefined"]
    cmd = [HIPCC, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-shared",
           "-fno-omit-frame-pointer", "-Wno-unused-command-line-argument",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"] + san + \
        [os.path.join(CSRC, s) for s in SOURCES] + ["-o", lib]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    exe = str(tmp_path / "host_driver")
    cmd = [CLANG, "-O1", "-g", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
           os.path.join(HERE, "sanitize", "host_driver.c"), lib,
           "-Wl,-rpath," + str(tmp_path), "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    # The HIP runtime the library links is not instrumented; its own allocations are not
    # this code's, so leak reports are off for this run.
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    res = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert res.returncode == 0, res.stdout + res.stderr
    assert "host driver ok" in res.stdout
    assert "runtime error" not in res.stderr and "AddressSanitizer" not in res.stderr, res.stderr
