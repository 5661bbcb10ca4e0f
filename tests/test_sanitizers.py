"""AddressSanitizer and UndefinedBehaviorSanitizer builds of the CPU code.

* the oracle (oracle/oracle.c) with gcc, driven by tests/sanitizers/oracle_check.c
  over small grids: every exported routine, preconditioner, face mask and the
  FP32 emulation, with complete solves;
* the library's host-side planning (paper_2503_08935_amd/csrc/plan.hip) with g++
  as host C++, driven by tests/sanitizers/plan_check.cpp with the kernel
  launchers replaced by recorders: the kernel sequence of an iteration over
  every plan, its byte count against the closed-form model, the workspace
  layout, the coefficients and the tilings.

Both programs exit 0 only if every check passes and no sanitizer fires.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitizers")
SAN = ["-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]


def run(exe, env_extra):
    env = dict(os.environ, **env_extra)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc missing")
def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_check")
    subprocess.check_call(["gcc"] + SAN + ["-fopenmp", "-ffp-contract=off",
                                           os.path.join(ROOT, "oracle", "oracle.c"),
                                           os.path.join(HERE, "oracle_check.c"), "-lm", "-o", exe])
    run(exe, {"OMP_NUM_THREADS": "2", "ASAN_OPTIONS": "detect_leaks=1"})


@pytest.mark.skipif(shutil.which("g++") is None or
                    not os.path.exists("/opt/rocm/include/hip/hip_runtime.h"),
                    reason="g++ or the HIP headers missing")
def test_host_planning_under_sanitizers(tmp_path):
    exe = str(tmp_path / "plan_check")
    csrc = os.path.join(ROOT, "paper_2503_08935_amd", "csrc")
    subprocess.check_call(["g++", "-std=c++17"] + SAN + [
        "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", "-I", os.path.join(ROOT, "include"),
        "-I", csrc, "-x", "c++", os.path.join(csrc, "plan.hip"),
        "-x", "c++", os.path.join(HERE, "plan_check.cpp"),
        "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib", "-o", exe])
    # the HIP runtime keeps allocations for the process lifetime: no leak check
    run(exe, {"ASAN_OPTIONS": "detect_leaks=0"})
