"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer (host
code, g++): oracle/sanitize_main.cpp calls every entry point of
oracle/oracle.cpp in every mode, with degenerate Gaussians, and any
out-of-bounds access, leak or undefined operation ends the run with a
report. CPU only."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_oracle_clean_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_sanitized")
    build = ["g++", "-O1", "-g", "-std=c++17", "-fopenmp", "-ffp-contract=off", "-fno-omit-frame-pointer",
             "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
             os.path.join(ROOT, "oracle", "oracle.cpp"), os.path.join(ROOT, "oracle", "sanitize_main.cpp"),
             "-o", exe]
    r = subprocess.run(build, capture_output=True, text=True, timeout=300)
    if r.returncode != 0 and "asan" in (r.stderr or "").lower():
        pytest.skip("sanitizer runtime not available: " + r.stderr[-300:])
    assert r.returncode == 0, r.stderr[-2000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", OMP_NUM_THREADS="2")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0 and "clean" in r.stdout, (r.stdout[-2000:], r.stderr[-4000:])
    assert "runtime error" not in r.stderr and "ERROR: AddressSanitizer" not in r.stderr, r.stderr[-4000:]
