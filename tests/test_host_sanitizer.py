"""The host side of the C ABI (argument validation, option parsing, error
strings, the tune-cache file parser) built from its C++ sources with g++
under AddressSanitizer and UndefinedBehaviorSanitizer and run without a GPU
(tests/host_sanitizer/driver.cpp).  Only host sources are compiled; the
device-side symbols those sources reference are left unresolved and never
called."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1805_09498_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None or not os.path.isdir("/opt/rocm/include"),
                    reason="needs g++ and the ROCm headers")
def test_host_layer_under_sanitizers(tmp_path):
    exe = tmp_path / "host_sanitizer"
    cmd = ["g++", "-std=c++17", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", "-I" + CSRC,
           "-I" + os.path.join(ROOT, "include"), "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-fno-omit-frame-pointer", "-g", "-O1", "-w",
           os.path.join(ROOT, "tests", "host_sanitizer", "driver.cpp"),
           os.path.join(CSRC, "fca_api.cpp"), os.path.join(CSRC, "fca_batch.cpp"),
           os.path.join(CSRC, "fca_tunecache.cpp"),
           "-L/opt/rocm/lib", "-lamdhip64", "-Wl,--unresolved-symbols=ignore-all", "-o", str(exe)]
    b = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert b.returncode == 0, b.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", HIP_VISIBLE_DEVICES="")
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0 and "HOST SANITIZER OK" in r.stdout, (r.stdout[-4000:], r.stderr[-4000:])
