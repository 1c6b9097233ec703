"""The library's host-side meshers and tuning-cache parser under the address
and undefined-behaviour sanitizers: tests/host_fuzz.cpp feeds them seeded
random valid and invalid inputs (boxes, partition rules, layered dielectric
layouts, truncated and corrupted cache files).  Host code only, built with
g++ (no device code is compiled); runs on the CPU."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2203_11733_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None or not os.path.isdir("/opt/rocm/include"),
                    reason="needs g++ and the ROCm headers")
def test_meshers_and_cache_parser_under_sanitizers(tmp_path):
    exe = str(tmp_path / "host_fuzz")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           "-fno-omit-frame-pointer", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", "-I", os.path.join(ROOT, "include"),
           "-I", CSRC, os.path.join(CSRC, "mesh.cpp"), os.path.join(CSRC, "tune.cpp"),
           os.path.join(ROOT, "tests", "host_fuzz.cpp"), "-ldl", "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe, "150"], capture_output=True, text=True, timeout=300, env=env)
    print(r.stdout[-2000:])
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert "0 inconsistencies" in r.stdout
