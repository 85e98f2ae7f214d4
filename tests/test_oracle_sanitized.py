"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer.

The oracle's C source is compiled for the host with -fsanitize=address,undefined
(no recovery: the first report aborts), and the whole oracle pin suite runs
against that build in a child process.  Out-of-bounds accesses, use after
free, signed overflow, overlong shifts and null arguments to libc (qsort with
an empty array) all end the run.  Host code only; the GPU library is not
involved.
"""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "sba_oracle.c")


def _runtime(name):
    p = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_suite_clean_under_sanitizers(tmp_path):
    asan = _runtime("libasan.so")
    if asan is None:
        pytest.skip("libasan runtime not installed")
    so = tmp_path / "liboracle_san.so"
    subprocess.run(["gcc", "-O1", "-g", "-fno-omit-frame-pointer",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                    "-std=gnu11", "-fopenmp", "-fPIC", "-shared", "-o", str(so), SRC, "-lm"],
                   check=True)
    env = dict(os.environ, ORACLE_LIBRARY=str(so), LD_PRELOAD=asan,
               ASAN_OPTIONS="detect_leaks=0", UBSAN_OPTIONS="print_stacktrace=1",
               OMP_NUM_THREADS="4")
    # -s: a sanitizer report is written to stderr just before the abort, so
    # pytest must not hold stderr back
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-s", "-p", "no:cacheprovider",
                        "-p", "no:xdist", os.path.join(ROOT, "tests", "test_oracle.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    out = r.stdout + r.stderr
    assert "runtime error" not in out and "AddressSanitizer" not in out, out[-3000:]
    assert r.returncode == 0, out[-3000:]
