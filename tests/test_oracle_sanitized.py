"""The oracle built with AddressSanitizer and UndefinedBehaviorSanitizer (gcc,
host code only) and run on seeded random inputs of many shapes through every
entry point (tests/sanitize/oracle_driver.c): any read or write outside the
arrays the header sizes, or undefined arithmetic, ends the run with an
error. The driver also checks that the OpenMP product equals the
single-threaded one and that malformed inputs are refused."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_under_asan_ubsan(tmp_path):
    exe = tmp_path / "oracle_driver"
    cmd = ["gcc", "-O1", "-g", "-std=c11", "-ffp-contract=off", "-fopenmp",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
           "-I", os.path.join(ROOT, "oracle"), "-o", str(exe),
           os.path.join(HERE, "sanitize", "oracle_driver.c"), os.path.join(ROOT, "oracle", "oracle.c")]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", OMP_NUM_THREADS="3")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "oracle driver: ok" in r.stdout
