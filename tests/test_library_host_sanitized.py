"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

Every source is rebuilt with the host half of each hipcc call instrumented (-Xarch_host before each
sanitizer flag; the gfx950 code is built as usual) into a temporary directory, and the host-only ABI
tests of tests/test_abi_cpu.py (argument validation, problem limits, workspace sizes and layouts,
error strings, thousands of hypothesis-drawn problems) run against that build in a subprocess through
PP_LIBRARY.  An out-of-bounds access, a use after free, a signed overflow or any other undefined
behaviour met on the way fails the run.  The sanitizer runtime is preloaded because the Python
interpreter is not instrumented; leak checking is off.
"""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN_FLAGS = ["-Xarch_host", "-fsanitize=address,undefined", "-Xarch_host", "-fno-sanitize-recover=all",
             "-Xarch_host", "-fno-omit-frame-pointer"]


def _asan_runtime():
    found = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return found[-1] if found else None


def test_abi_host_code_under_sanitizers(tmp_path):
    rt = _asan_runtime()
    if rt is None:
        pytest.skip("the ROCm clang has no AddressSanitizer runtime here")
    sys.path.insert(0, ROOT)
    from paper_2307_12041_amd import build
    lib = build.build(out_path=str(tmp_path / "libpplace_san.so"), build_dir=str(tmp_path / "obj"),
                      extra_flags=SAN_FLAGS)
    probe = subprocess.run(["nm", "-D", lib], capture_output=True, text=True)
    assert "__asan_report" in probe.stdout, "the host code of the rebuilt library is not instrumented"
    env = dict(os.environ, PP_LIBRARY=lib, LD_PRELOAD=rt,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_abi_cpu.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=1200)
    assert r.returncode == 0, f"ABI tests failed on the sanitized library:\n{r.stdout[-3000:]}\n{r.stderr[-3000:]}"
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-3000:]
