"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU
only): the library's planning and schedule entry points (csrc/sk_api.hip
host code, driven by tests/sanitize/host_abi_driver.cpp with a hand-made
tile registry) and the oracle's FP64 GEMM (oracle/gemm_f64.c, driven by
tests/sanitize/oracle_driver.c).  Device code is compiled without
instrumentation (the sanitizer flags apply to the host pass only)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
BUILD = os.path.join(ROOT, "_build", "sanitize")
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
           UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout}\n{r.stderr}"
    return r


@pytest.mark.skipif(not os.path.exists("/opt/rocm/bin/hipcc"), reason="needs hipcc")
def test_host_library_code_under_asan_ubsan():
    os.makedirs(BUILD, exist_ok=True)
    exe = os.path.join(BUILD, "host_abi_driver")
    san = ["-Xarch_host", "-fsanitize=address,undefined", "-Xarch_host", "-fno-omit-frame-pointer"]
    _run(["/opt/rocm/bin/hipcc", "--offload-arch=gfx950", "-O1", "-g", "-std=c++17",
          "-Wno-unused-command-line-argument", "-Xclang", "-target-feature", "-Xclang",
          "-packed-fp32-ops", "-I" + os.path.join(ROOT, "include")] + san +
         [os.path.join(HERE, "host_abi_driver.cpp"),
          os.path.join(ROOT, "paper_2407_00044_amd", "csrc", "sk_api.hip"),
          os.path.join(ROOT, "paper_2407_00044_amd", "csrc", "sk_transpose.hip"), "-o", exe])
    r = _run([exe], env=ENV, timeout=300)
    assert "host ABI driver: ok" in r.stdout
    assert "runtime error" not in r.stderr


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_gemm_under_asan_ubsan():
    os.makedirs(BUILD, exist_ok=True)
    exe = os.path.join(BUILD, "oracle_driver")
    _run(["gcc", "-O1", "-g", "-std=c11", "-fopenmp", "-ffp-contract=off",
          "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
          os.path.join(HERE, "oracle_driver.c"), os.path.join(ROOT, "oracle", "gemm_f64.c"),
          "-o", exe])
    r = _run([exe], env=dict(ENV, OMP_NUM_THREADS="4"), timeout=300)
    assert "oracle driver: ok" in r.stdout
    assert "runtime error" not in r.stderr
