"""The host half of the library (api.cpp, lgl.cpp) built with g++ under
AddressSanitizer and UndefinedBehaviorSanitizer and driven through its C ABI
on the CPU (tests/sanitize/host_driver.cpp): LGL tables, validation, host
copies of the mesh arrays, workspace sizing and the pre-bind state errors.
The kernel launchers are stubs that abort if reached."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2606_18927_amd", "csrc")
HIP = "/opt/rocm"


@pytest.mark.skipif(shutil.which("g++") is None or not os.path.exists(os.path.join(HIP, "lib", "libamdhip64.so")),
                    reason="needs g++ and the HIP runtime library")
def test_host_paths_under_asan_ubsan(tmp_path):
    exe = tmp_path / "host_driver"
    cmd = ["g++", "-std=c++17", "-g", "-O1", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-D__HIP_PLATFORM_AMD__", f"-I{HIP}/include",
           os.path.join(CSRC, "api.cpp"), os.path.join(CSRC, "lgl.cpp"),
           os.path.join(ROOT, "tests", "sanitize", "launch_stubs.cpp"),
           os.path.join(ROOT, "tests", "sanitize", "host_driver.cpp"),
           f"-L{HIP}/lib", "-lamdhip64", f"-Wl,-rpath,{HIP}/lib", "-o", str(exe)]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    run = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300, env=env)
    assert run.returncode == 0, (run.stdout[-2000:], run.stderr[-4000:])
    assert "all expectations hold" in run.stdout
