"""The host ABI layer (validation, layout, error strings, NULL handling)
built with AddressSanitizer, LeakSanitizer and UndefinedBehaviorSanitizer
and run on the CPU: tests/host_abi/abi_check.cpp drives every entry point
on paths that need no device, with the device-side launch helpers replaced
by stand-ins that abort if reached (tests/host_abi/launch_stubs.cpp)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1904_08463_amd", "csrc")
HERE = os.path.join(ROOT, "tests", "host_abi")


@pytest.mark.skipif(shutil.which("g++") is None or not os.path.isdir("/opt/rocm/include"),
                    reason="needs g++ and the ROCm headers")
def test_host_abi_under_sanitizers(tmp_path):
    exe = str(tmp_path / "abi_check")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
           f"-I{os.path.join(ROOT, 'include')}", f"-I{CSRC}",
           os.path.join(CSRC, "wkern.cpp"), os.path.join(HERE, "launch_stubs.cpp"),
           os.path.join(HERE, "abi_check.cpp"),
           "-L/opt/rocm/lib", "-lamdhip64", "-lrocprofiler-sdk-roctx", "-Wl,-rpath,/opt/rocm/lib",
           "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1",
               HIP_VISIBLE_DEVICES="", WKERN_FAULT="", WKERN_LOG="0")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, (r.stdout + r.stderr)[-4000:]
    assert "host ABI checks passed" in r.stdout
