"""The host grid builder (C++) under AddressSanitizer and
UndefinedBehaviorSanitizer: every grid entry point on levels 0-4, standard
and smoothed, and the argument checks, with any report failing the test."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_grid_builder_is_clean_under_sanitizers(tmp_path):
    exe = str(tmp_path / "grid_sanitize")
    src = os.path.join(ROOT, "paper_1607_05535_amd", "csrc", "grid.cpp")
    drv = os.path.join(ROOT, "tests", "native", "grid_sanitize_driver.cpp")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-pthread",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           "-I", os.path.join(ROOT, "paper_1607_05535_amd", "csrc"), src, drv, "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, timeout=300)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "runtime error" not in r.stderr and "ERROR: AddressSanitizer" not in r.stderr
    assert r.stdout.strip().endswith("ok")
