"""The oracle's C and the library's host C++ (code construction, decode-table
build, argument checks and job tables of every entry point) built for the CPU
with AddressSanitizer and UndefinedBehaviorSanitizer (g++/gcc, no device
code: the kernel launchers are stand-ins that report a runtime error) and run
on random and edge-case inputs by tests/sanitize/host_checks.cpp."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ROCM_INCLUDE = "/opt/rocm/include"
ROCM_LIB = "/opt/rocm/lib"
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]


def test_host_code_under_sanitizers(tmp_path):
    if not shutil.which("g++") or not os.path.isdir(ROCM_INCLUDE):
        pytest.skip("g++ or the HIP headers are missing")
    oracle_o = tmp_path / "oracle.o"
    subprocess.run(["gcc", "-std=c99", *SAN, "-c", os.path.join(ROOT, "oracle", "hc_oracle.c"), "-o", str(oracle_o)],
                   check=True)
    exe = tmp_path / "host_checks"
    csrc = os.path.join(ROOT, "paper_1107_1525_amd", "csrc")
    subprocess.run(
        ["g++", "-std=c++17", *SAN, "-D__HIP_PLATFORM_AMD__", "-I", ROCM_INCLUDE, "-I", os.path.join(ROOT, "include"),
         "-I", csrc, os.path.join(csrc, "hc_api.cpp"), os.path.join(csrc, "hc_codebook.cpp"),
         os.path.join(ROOT, "tests", "sanitize", "launch_stubs.cpp"),
         os.path.join(ROOT, "tests", "sanitize", "host_checks.cpp"), str(oracle_o),
         "-L", ROCM_LIB, "-Wl,-rpath," + ROCM_LIB, "-lamdhip64", "-lpthread", "-o", str(exe)],
        check=True)
    env = dict(os.environ)
    # the HIP runtime library is not instrumented and keeps allocations for the process
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    env["HIP_VISIBLE_DEVICES"] = ""
    res = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=600)
    assert res.returncode == 0, res.stdout + res.stderr
    assert "host checks OK" in res.stdout
