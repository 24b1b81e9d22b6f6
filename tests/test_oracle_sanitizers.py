"""The CPU oracle under AddressSanitizer (with leak checks) and
UndefinedBehaviorSanitizer: tests/oracle_sanitize_main.cpp, built with g++
on the host only, runs every oracle entry point on small seeded states
(every boundary type on every side, both orders, the three fluxes, the
friction laws, rain and soil fields, a hyetograph, the tangent and gauge
runs).  Any invalid access or undefined operation aborts the run."""

import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_oracle_clean_under_sanitizers(tmp_path):
    exe = str(tmp_path / "orc_san")
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-g", "-fopenmp", "-ffp-contract=off",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                           "-fno-omit-frame-pointer",
                           os.path.join(HERE, "oracle_sanitize_main.cpp"), "-o", exe])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1", OMP_NUM_THREADS="2")
    r = subprocess.run([exe], env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "0 failures" in r.stdout
