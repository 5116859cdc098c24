"""The C ABI from a plain C++ caller (tests/c_abi/abi_caller.cpp): HIP runtime allocations and
stream, pp_workspace_size, pp_energy and pp_field, no Python binding and no torch on the path,
against the FP64 oracle (whole arrays and worst tiles of the flat-spectrum raw sums and of the
gradient).  The caller is a shared library built by build() and driven in-process."""
import ctypes
import os
import sys

import numpy as np
import pytest

import oracle
from tests import parity
from workloads import make_random

pytestmark = pytest.mark.gpu
LIB = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c_abi", "libabi_caller.so")
PREC = {"fp64": (0, 1e-10), "fp32": (1, 1e-5), "bf16x3": (3, 1e-3)}


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def rel(a, b):
    nb = np.linalg.norm(np.ravel(b))
    return np.linalg.norm(np.ravel(a) - np.ravel(b)) / (nb if nb > 0 else 1.0)


@pytest.fixture(scope="module")
def caller():
    if not os.path.exists(LIB):
        raise RuntimeError(f"{LIB} is not built; run `python -c 'import __graft_entry__ as g; g.build()'`")
    lib = ctypes.CDLL(LIB)
    d, dp = ctypes.c_double, ctypes.POINTER(ctypes.c_double)
    lib.abi_caller_run.argtypes = [d, d, ctypes.c_int64, ctypes.c_int, ctypes.c_int, ctypes.c_int, dp, dp, dp, dp,
                                   dp, dp, dp, dp, ctypes.c_char_p, ctypes.c_int]
    lib.abi_caller_run.restype = ctypes.c_int
    return lib


def call(lib, wl, prec):
    arrs = [np.ascontiguousarray(v, dtype=np.float64) for v in wl.arrays()]
    E = np.zeros(1)
    a = np.zeros((wl.Mu, wl.Mp))
    gx, gy = np.zeros(wl.n), np.zeros(wl.n)
    msg = ctypes.create_string_buffer(256)
    ptr = lambda v: v.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    st = lib.abi_caller_run(wl.W, wl.H, wl.n, wl.Mu, wl.Mp, PREC[prec][0], *[ptr(v) for v in arrs], ptr(E), ptr(a),
                            ptr(gx), ptr(gy), msg, 256)
    return st, msg.value.decode(), float(E[0]), a, gx, gy


@pytest.mark.parametrize("prec", sorted(PREC))
def test_plain_cpp_caller_matches_oracle(caller, prec):
    wl = make_random(1537, 300.0, 170.0, 131, 77, seed=71)
    say(f"[c caller] {prec} n={wl.n} M={wl.Mu}x{wl.Mp}")
    st, msg, E, a, gx, gy = call(caller, wl, prec)
    assert st == 0, msg
    Eo, ao, _ = oracle.energy(wl.W, wl.H, *wl.arrays(), wl.Mu, wl.Mp)
    gxo, gyo = oracle.grad(wl.W, wl.H, *wl.arrays(), ao)
    f = oracle.coef_factors(wl.W, wl.H, wl.Mu, wl.Mp)
    ce = parity.coeff_errors(a, parity.raw_from_coeffs(ao, f), f)
    g, go = np.stack([gx, gy], axis=1), np.stack([gxo, gyo], axis=1)
    errs = (abs(E - Eo) / Eo, rel(a, ao), ce["flat"], ce["flat_tile"], rel(g, go), parity.row_tile_rel_max(g, go))
    say(f"   E {errs[0]:.2e}  a {errs[1]:.2e}  flat a {errs[2]:.2e} (worst 64x64 tile {errs[3]:.2e})  "
        f"g {errs[4]:.2e} (worst 256-block tile {errs[5]:.2e})")
    assert max(errs) <= PREC[prec][1], errs


def test_plain_cpp_caller_reports_errors(caller):
    wl = make_random(10, 30.0, 20.0, 5, 5, seed=72)
    wl.Mu = 0
    st, msg, *_ = call(caller, wl, "fp64")
    assert st == -1 and "pp_workspace_size" in msg
