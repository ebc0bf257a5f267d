"""AddressSanitizer / UndefinedBehaviorSanitizer builds of the host code.

The FP64 oracle (``oracle/lbm_oracle.c``) and the GPU library's host geometry
(``csrc/geometry.cpp``: voxelisation, wall links, wall distances, flag words)
are compiled with ``-fsanitize=address,undefined`` into two small driver
programs under ``tests/sanitize/`` that call every entry point on random
inputs, including one-cell edges and fully periodic sphere images.  Any
out-of-bounds access, leak or undefined operation makes the driver exit with a
non-zero status.  CPU only: no GPU code is built with a sanitizer.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
       "-fno-omit-frame-pointer"]


def _run(cmd, exe, tmp_path):
    subprocess.run(cmd, check=True, cwd=ROOT)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    env.pop("LD_PRELOAD", None)
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "0 failures" in r.stdout


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_driver")
    cmd = ["gcc", *SAN, "-std=c99", "-ffp-contract=off", "-I", "oracle", "-o", exe,
           "tests/sanitize/oracle_driver.c", "oracle/lbm_oracle.c", "-lm"]
    _run(cmd, exe, tmp_path)


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_host_geometry_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "geometry_driver")
    cmd = ["g++", *SAN, "-std=c++17", "-I", "include", "-I", "paper_1508_02960_amd/csrc",
           "-o", exe, "tests/sanitize/geometry_driver.cpp",
           "paper_1508_02960_amd/csrc/geometry.cpp", "-lpthread"]
    _run(cmd, exe, tmp_path)
