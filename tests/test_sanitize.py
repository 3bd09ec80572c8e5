"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

* the C ABI's host half (``csrc/abi.cpp``: validation, workspace layout, fan
  tables, plan bookkeeping) linked with host-only stand-ins for the HIP
  runtime and the kernel launchers (``tests/sanitize/abi_stubs.cpp``), driven
  through every entry point with valid and invalid arguments;
* the FP64 oracle (``oracle/diffus_oracle.c``) on small inputs that cover
  clamped samples, both reflection conventions, every attenuation mode,
  speckle and blur, and the edge sizes.

Any sanitizer report aborts the program (``-fno-sanitize-recover=all``).
Device code is not built here: GPU sanitizers are not used.
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SAN = ["-g", "-O1", "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]


def _run(cmd_build, exe):
    subprocess.check_call(cmd_build)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    env.pop("LD_PRELOAD", None)
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr
    return r.stdout


def test_abi_host_code_sanitized(tmp_path):
    gxx = shutil.which("g++")
    if not gxx or not os.path.exists("/opt/rocm/include/hip/hip_runtime_api.h"):
        pytest.skip("g++ or the HIP headers are not available")
    exe = str(tmp_path / "abi_driver")
    out = _run([gxx, "-std=c++17", *SAN, "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", "-o", exe,
                os.path.join(HERE, "sanitize", "abi_driver.cpp"), os.path.join(HERE, "sanitize", "abi_stubs.cpp"),
                os.path.join(ROOT, "paper_2508_06768_amd", "csrc", "abi.cpp")], exe)
    assert "abi driver: ok" in out


def test_oracle_sanitized(tmp_path):
    gcc = shutil.which("gcc")
    if not gcc:
        pytest.skip("gcc is not available")
    exe = str(tmp_path / "oracle_driver")
    out = _run([gcc, "-std=gnu99", *SAN, "-ffp-contract=off", "-o", exe,
                os.path.join(HERE, "sanitize", "oracle_driver.c"), "-lm"], exe)
    assert "oracle driver: ok" in out
