"""The oracle under the host sanitizers: tests/oracle_sanitized/driver.c, which calls every
entry point of oracle/ora.h on small 2D and 3D grids with every boundary kind, marker motion,
scheme and reconstruction variable, is built together with oracle/ora.c with gcc's
AddressSanitizer (bounds, use after free, leaks) and UndefinedBehaviorSanitizer, and must run
clean. The oracle is test infrastructure; this keeps the code the GPU path is checked against
free of memory errors that could make it compute something other than what it reads as.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_oracle_runs_clean_under_asan_and_ubsan(tmp_path):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no gcc")
    exe = str(tmp_path / "ora_sanitized")
    build = [gcc, "-std=c11", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
             "-fno-sanitize-recover=all", "-fopenmp", "-I", os.path.join(ROOT, "oracle"),
             os.path.join(ROOT, "tests", "oracle_sanitized", "driver.c"), os.path.join(ROOT, "oracle", "ora.c"),
             "-lm", "-o", exe]
    r = subprocess.run(build, capture_output=True, text=True)
    if r.returncode != 0 and "asan" in (r.stderr or "").lower():
        pytest.skip("the sanitizer runtimes are not installed: " + r.stderr[-300:])
    assert r.returncode == 0, r.stderr
    # (verify_asan_link_order=0: the environment may preload a library of its own ahead of the
    # sanitizer runtime)
    env = dict(os.environ, OMP_NUM_THREADS="1",
               ASAN_OPTIONS="detect_leaks=1:abort_on_error=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert "ran clean" in r.stdout
