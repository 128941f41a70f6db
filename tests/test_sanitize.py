"""Host sanitizer runs (no GPU): the C oracle and the library's host-only plan
code, each built on its own with AddressSanitizer and UBSan (gcc / g++) and
driven over small inputs, error paths and extreme arguments by the drivers in
tests/sanitize/.  Any out-of-bounds access, leak, overflow or undefined
operation aborts the driver."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
SAN = ["-g", "-O1", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
       "-fno-omit-frame-pointer"]


def _run(exe):
    env = dict(os.environ, ASAN_OPTIONS="abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    print(r.stdout, r.stderr)
    return r


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_san")
    subprocess.check_call(["gcc", "-std=c11", *SAN, os.path.join(HERE, "oracle_driver.c"),
                           os.path.join(ROOT, "oracle", "cdmt_oracle.c"), "-o", exe, "-lm",
                           "-lpthread"])
    r = _run(exe)
    assert r.returncode == 0 and "ok" in r.stdout


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_plan_code_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "plan_san")
    subprocess.check_call(["g++", "-std=c++17", *SAN, "-I", os.path.join(ROOT, "include"),
                           os.path.join(HERE, "plan_driver.cpp"),
                           os.path.join(ROOT, "paper_1607_00909_amd", "csrc", "plan.cpp"),
                           "-o", exe])
    r = _run(exe)
    assert r.returncode == 0 and "ok" in r.stdout
