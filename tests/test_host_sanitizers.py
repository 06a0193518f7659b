"""The library's host-only code (canonicalisation with its smallest-circle and
equilibration routines, the pantograph gather, the Jacobi eigensolver) built
with g++ under AddressSanitizer and UndefinedBehaviorSanitizer and run on
random and degenerate inputs (no GPU involved)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_host_code_under_address_and_ub_sanitizers(tmp_path):
    exe = tmp_path / "sanitize_driver"
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined",
           os.path.join(ROOT, "tests", "host", "sanitize_driver.cpp"),
           os.path.join(ROOT, "paper_2207_14222_amd", "csrc", "canon.cpp"), "-o", str(exe)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    # verify_asan_link_order=0: the environment may preload a library ahead of
    # the sanitizer runtime, which is harmless here
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert "0 failures" in r.stdout
