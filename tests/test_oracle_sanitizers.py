"""The C oracle built with AddressSanitizer and UndefinedBehaviorSanitizer (host gcc) and run
through every entry point on small lattice inputs (tests/oracle_sanitize_driver.c): no
out-of-bounds access, leak or undefined arithmetic."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc is not installed")
def test_oracle_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_sanitize")
    cmd = ["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-fno-fast-math", "-ffp-contract=off", "-fopenmp", "-std=c11",
           "-D_GNU_SOURCE", "-o", exe, os.path.join(HERE, "oracle_sanitize_driver.c"),
           os.path.join(ROOT, "oracle", "aidw_oracle.c"), "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0 and "asan" in (r.stderr + r.stdout).lower():
        pytest.skip("the sanitizer runtime is not available: " + r.stderr[-300:])
    assert r.returncode == 0, r.stderr
    env = dict(os.environ, OMP_NUM_THREADS="4", ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    run = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert "runtime error" not in run.stderr, run.stderr[-2000:]
    assert "AddressSanitizer" not in run.stderr, run.stderr[-2000:]
    assert run.returncode == 0, run.stderr[-2000:]
