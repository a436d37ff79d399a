"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

* The HIP-free argument checks and tile planning of the library
  (paper_1210_3165_amd/csrc/bz_host.hpp, the code every entry point runs
  before a launch) built with g++ into a driver that compares the strided
  alias test with brute force and checks the parameter range, decision
  constants, image checks and default tiles.
* The C oracle built with gcc, driven over every small shape, window and
  entry point.
Both are built here with -fsanitize=address,undefined and must run clean.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
NATIVE = os.path.join(ROOT, "tests", "native")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]


def _build_and_run(tmp_path, cmd, exe):
    res = subprocess.run(cmd, capture_output=True, text=True)
    assert res.returncode == 0, res.stdout + res.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    run = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert run.returncode == 0, run.stdout[-4000:] + run.stderr[-4000:]
    return run.stdout


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ missing")
def test_host_checks_under_sanitizers(tmp_path):
    exe = str(tmp_path / "host_checks")
    cmd = ["g++", "-std=c++17", *SAN, "-I", os.path.join(ROOT, "include"),
           "-I", os.path.join(ROOT, "paper_1210_3165_amd", "csrc"),
           os.path.join(NATIVE, "host_checks.cpp"), "-o", exe]
    out = _build_and_run(tmp_path, cmd, exe)
    assert "host checks passed" in out


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc missing")
def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_drive")
    cmd = ["gcc", "-std=c99", *SAN, os.path.join(ROOT, "oracle", "oracle.c"),
           os.path.join(NATIVE, "oracle_drive.c"), "-lm", "-o", exe]
    out = _build_and_run(tmp_path, cmd, exe)
    assert "ok" in out
