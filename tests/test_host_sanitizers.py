"""The library's host code (schedule designer, grid checks, dense exponential,
checkpoint reader, autotuner cache) built with g++ under AddressSanitizer and UndefinedBehaviour
Sanitizer and run on valid and invalid inputs (no GPU)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2506_03617_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ is not available")
def test_host_code_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    exe = str(tmp_path / "sanitize_host")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-I", os.path.join(ROOT, "include"),
           os.path.join(ROOT, "tests", "sanitize_host.cpp"),
           os.path.join(CSRC, "schedule.cpp"), os.path.join(CSRC, "checkpoint.cpp"),
           os.path.join(CSRC, "tunecache.cpp"), "-o", exe]
    subprocess.run(cmd, check=True, timeout=300)
    # a library preloaded into every process may come before the sanitizer runtime
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe, str(tmp_path)], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "all host checks passed" in r.stdout
    assert "runtime error" not in r.stderr
