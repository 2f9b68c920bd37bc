"""Host-side AddressSanitizer / UndefinedBehaviorSanitizer run of the C
oracles: tests/sanitize/oracle_sanitize_main.c calls every exported function
of oracle/tnlm_oracle.c and oracle/ct_oracle.c on small awkward grids; the
three files are built with gcc (no OpenMP) and any sanitizer report fails
the test."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SOURCES = [os.path.join(ROOT, p) for p in (
    "tests/sanitize/oracle_sanitize_main.c", "oracle/tnlm_oracle.c", "oracle/ct_oracle.c")]


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not installed")
def test_oracle_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_sanitize")
    cmd = ["gcc", "-std=c99", "-g", "-O1", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined,float-cast-overflow",
           "-fno-sanitize-recover=all", "-Wall", "-Wno-unknown-pragmas",
           "-o", exe, *SOURCES, "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0 and ("libasan" in r.stderr or "libubsan" in r.stderr):
        pytest.skip("gcc has no sanitizer runtime here: " + r.stderr[-200:])
    assert r.returncode == 0, r.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    run = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert run.returncode == 0, run.stdout + run.stderr
    assert "runtime error" not in run.stderr and "Sanitizer" not in run.stderr, run.stderr
    assert "all cases passed" in run.stdout
