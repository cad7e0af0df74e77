"""The host set-up (host_setup.cpp: splines, quadrature points and weights for
both rules, geometry, eigenpairs) built with g++ under AddressSanitizer and
UndefinedBehaviorSanitizer and run over p = 2..10 (tests/host_setup_driver.cpp).
CPU only; skipped when g++ is missing."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_host_setup_under_address_and_ub_sanitizers(tmp_path):
    exe = str(tmp_path / "host_setup_driver")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-fno-omit-frame-pointer", "-pthread", "-I", os.path.join(ROOT, "include"),
           os.path.join(ROOT, "tests", "host_setup_driver.cpp"),
           os.path.join(ROOT, "paper_1712_08565_amd", "csrc", "host_setup.cpp"), "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, timeout=300)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0 and "ok" in r.stdout, (r.returncode, r.stdout[-2000:], r.stderr[-4000:])
