"""Sanitizer builds of the host code that runs without a GPU: the CPU oracle (through
tests/sanitize_oracle.c) and the library's host logic of the symbolic phase (tiles, table
capacities, the hash multiplier; through tests/host_logic_check.cpp), each compiled with gcc's
AddressSanitizer and UndefinedBehaviorSanitizer and run to completion.  Any out-of-bounds access,
use after free, leak or undefined behaviour makes the run fail."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
FLAGS = ["-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
         "-fno-omit-frame-pointer"]


def _run(cmd, exe, tmp_path):
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "runtime error" not in r.stderr and "ERROR: AddressSanitizer" not in r.stderr, r.stderr[-4000:]
    return r.stdout


def test_oracle_under_sanitizers(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    exe = str(tmp_path / "sanitize_oracle")
    out = _run(["gcc", *FLAGS, "-std=c11", "-pthread", os.path.join(HERE, "sanitize_oracle.c"),
                os.path.join(ROOT, "oracle", "ptap_oracle.c"), "-lm", "-o", exe], exe, tmp_path)
    assert out.strip().endswith("ok")


def test_host_logic_under_sanitizers(tmp_path):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path / "host_logic_check")
    out = _run(["g++", *FLAGS, "-std=c++17", "-pthread", os.path.join(HERE, "host_logic_check.cpp"),
                "-o", exe], exe, tmp_path)
    assert "FAIL" not in out and "ok tiles 27pt_64" in out
