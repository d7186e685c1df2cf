"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer.

tests/sanitize/oracle_sanitize.c drives every entry point of
oracle/cps_oracle.c on small grids that reach its edge cases (ragged dims,
the full sphere's polar faces, every map and metric method, every outer
iteration, the projection step and the line solves).  It is built here with
gcc and the sanitizers, run on two OpenMP threads, and must finish without a
report: memory errors, leaks and undefined behaviour all abort the run."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_clean_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_sanitize")
    src = os.path.join(HERE, "sanitize", "oracle_sanitize.c")
    subprocess.check_call(["gcc", "-std=c11", "-O1", "-g", "-fno-omit-frame-pointer", "-fopenmp",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                           "-o", exe, src, "-lm"])
    env = dict(os.environ, OMP_NUM_THREADS="2",
               ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:exitcode=23:"
                            "verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1:exitcode=24")
    r = subprocess.run([exe], env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, (r.returncode, r.stderr[-4000:])
    assert "oracle sanitize: ok" in r.stdout
