"""The serving scheduler's admission policy on the CPU: tests/sched_mock.cpp
runs the library's own policy code (csrc/admission.h, the template the
scheduler thread calls) over a mock executor: simulated workers whose
workspaces grow per buffer and persist between jobs, jobs that finish while
idle workspaces are being freed, queued jobs withdrawn meanwhile, and seeded
random job streams.  It checks that what the device may hold never exceeds
the budget, that a starving head is never passed, that a blocked head is
passed while it is not starving, that idle workspaces are released when in
the way, and that every job runs.  Built with g++ under the address and
undefined-behaviour sanitizers; no device code."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2203_11733_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_admission_policy_with_mock_executor(tmp_path):
    exe = str(tmp_path / "sched_mock")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-Wall", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           "-fno-omit-frame-pointer", "-I", CSRC, os.path.join(ROOT, "tests", "sched_mock.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe, "300"], capture_output=True, text=True, timeout=300, env=env)
    print(r.stdout[-2000:])
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert " 0 violations" in r.stdout
