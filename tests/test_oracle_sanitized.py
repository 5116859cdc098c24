"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

The oracle's C source is built with -fsanitize=address,undefined (every report fatal) and the
whole pin suite runs against that build in a subprocess, through PP_ORACLE_LIB.  An out-of-bounds
access, a use after free, a signed overflow or any other undefined behaviour met on the way fails
the run.  The sanitizer runtime is preloaded because the Python interpreter itself is not
instrumented; leak checking is off (the interpreter keeps its own allocations to the end).
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "pp_oracle.c")


def _runtime(name):
    path = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


def test_pins_pass_on_the_sanitized_oracle(tmp_path):
    asan = _runtime("libasan.so")
    if asan is None:
        pytest.skip("gcc has no AddressSanitizer runtime here")
    lib = tmp_path / "liboracle_asan.so"
    subprocess.run(["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=all", "-fopenmp", "-fPIC", "-shared", "-std=c11", SRC, "-o", str(lib),
                    "-lm"], check=True)
    env = dict(os.environ, PP_ORACLE_LIB=str(lib), OMP_NUM_THREADS="4", LD_PRELOAD=asan,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=1200)
    assert r.returncode == 0, f"pins failed on the sanitized oracle:\n{r.stdout[-3000:]}\n{r.stderr[-3000:]}"
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-3000:]
