"""The host-side plan set-up (descriptor validation, stability bound, PML
factors, sensor CSR tables and their transpose) built on its own with g++
under AddressSanitizer and UndefinedBehaviorSanitizer and exercised over
valid, broken, edge and random inputs (tests/host_check.cpp).  Host code
only: no HIP header, no device."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1603_02329_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_host_plan_code_is_clean_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "host_check")
    flags = ["-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
             "-fno-sanitize-recover=all", "-I", os.path.join(ROOT, "include")]
    cmd = ["g++", *flags, os.path.join(ROOT, "tests", "host_check.cpp"), os.path.join(CSRC, "host_plan.cpp"),
           "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, (r.stdout[-4000:], r.stderr[-4000:])
    assert "all checks passed" in r.stdout
