"""The C ABI on the host (CPU only): the library loads, exports exactly what include/pplace.h
declares, sizes workspaces, and rejects bad arguments before touching the device.  No call here
reaches a kernel launch."""
import ctypes
import math
import os
import re
import subprocess

import pytest

import paper_2307_12041_amd as pp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pplace.h")


def header_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(pp_[a-z_0-9]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(pp.library_path()):
        pytest.skip("libpplace.so not built")
    return pp.load()


def test_exports_match_header(lib):
    declared = header_functions()
    assert set(pp.EXPORTS) <= set(declared)
    out = subprocess.run(["nm", "-D", "--defined-only", pp.library_path()], capture_output=True, text=True,
                         check=True).stdout
    exported = sorted(set(re.findall(r"\bT (pp_[a-z_0-9]+)$", out, flags=re.M)))
    assert exported == declared
    for f in declared:
        assert hasattr(lib, f)


def test_strerror(lib):
    for st in (0, -1, -2, -3, -4, -5, 7):
        s = lib.pp_strerror(st)
        assert isinstance(s, bytes) and len(s) > 3


def test_mfma_calibrate_rejects_bad_arguments_before_launch(lib):
    """The calibration hook validates on the host: no launch (none could run here) for a workgroup
    count outside 1..65535, an iteration count below 1 or a NULL output."""
    buf = ctypes.c_void_p(0x1000)   # never dereferenced: every call below must fail validation
    for wg, it, out in ((0, 10, buf), (65536, 10, buf), (-3, 10, buf), (256, 0, buf), (256, -1, buf),
                        (256, 10, None)):
        assert lib.pp_mfma_calibrate(wg, it, out, None) == -1


def P(**kw):
    d = dict(W=100.0, H=50.0, n=1000, Mu=64, Mp=48, precision=0, basis_mode=0)
    d.update(kw)
    return pp.PPProblem(d["W"], d["H"], d["n"], d["Mu"], d["Mp"], d["precision"], d["basis_mode"])


def ws_size(lib, prob):
    out = ctypes.c_size_t(12345)
    st = lib.pp_workspace_size(ctypes.byref(prob), ctypes.byref(out))
    return st, out.value


def test_limits_are_inclusive(lib):
    """The largest documented problems are accepted (their grids fit): n = 2^31 - 512 blocks,
    Mu * Mp = 2^30 frequency pairs, and the largest stored-basis problem of one shape."""
    for prec in (0, 1, 2, 3):
        assert ws_size(lib, P(n=2 ** 31 - 512, precision=prec))[0] == 0
        assert ws_size(lib, P(Mu=65536, Mp=16384, precision=prec))[0] == 0
        assert ws_size(lib, P(Mu=32768, Mp=32768, precision=prec, n=100))[0] == 0
    assert ws_size(lib, P(precision=3, basis_mode=1, n=256 * (2 ** 21 // 4 - 1), Mu=1024, Mp=8))[0] == 0


def test_workspace_size_monotone_and_host_only(lib):
    st, a = ws_size(lib, P(n=1000))
    assert st == 0 and a > 0 and a % 256 == 0
    st, b = ws_size(lib, P(n=100000))
    assert st == 0 and b >= a
    st, c = ws_size(lib, P(n=0))
    assert st == 0
    st, d = ws_size(lib, P(Mu=2048, Mp=2048, n=2_000_500))
    assert st == 0 and d > b


@pytest.mark.parametrize("bad,code", [
    (dict(W=0.0), -1), (dict(W=-1.0), -1), (dict(H=math.nan), -1), (dict(W=math.inf), -1),
    (dict(Mu=0), -1), (dict(Mp=-3), -1), (dict(Mu=70000), -1), (dict(n=-1), -1),
    (dict(precision=9), -1), (dict(basis_mode=5), -1),
    (dict(n=2 ** 31 - 511), -1), (dict(Mu=65536, Mp=16385), -1), (dict(Mu=32768, Mp=32769), -1),
    (dict(precision=3, basis_mode=1, n=2 ** 29, Mu=1024, Mp=8), -1),
])
def test_workspace_size_rejects(lib, bad, code):
    st, v = ws_size(lib, P(**bad))
    assert st == code and v == 12345      # output untouched


def test_entry_points_validate_before_launch(lib):
    prob = P()
    st, need = ws_size(lib, prob)
    assert st == 0
    fake = ctypes.c_void_p(1 << 20)      # never dereferenced: every call below fails validation
    nul = None
    # NULL problem
    assert lib.pp_coeffs(None, fake, fake, fake, fake, fake, fake, need, nul) == -1
    # NULL block arrays / outputs
    assert lib.pp_coeffs(ctypes.byref(prob), nul, fake, fake, fake, fake, fake, need, nul) == -1
    assert lib.pp_coeffs(ctypes.byref(prob), fake, fake, fake, fake, nul, fake, need, nul) == -1
    assert lib.pp_energy(ctypes.byref(prob), fake, fake, fake, fake, nul, fake, fake, need, nul) == -1
    assert lib.pp_field(ctypes.byref(prob), fake, fake, fake, fake, nul, nul, fake, fake, fake, need, nul) == -1
    assert lib.pp_field(ctypes.byref(prob), fake, fake, fake, fake, fake, nul, nul, fake, fake, need, nul) == -1
    # misaligned pointers
    odd = ctypes.c_void_p((1 << 20) + 4)
    assert lib.pp_coeffs(ctypes.byref(prob), odd, fake, fake, fake, fake, fake, need, nul) == -1
    # short / missing / misaligned workspace
    assert lib.pp_coeffs(ctypes.byref(prob), fake, fake, fake, fake, fake, fake, need - 1, nul) == -2
    assert lib.pp_energy(ctypes.byref(prob), fake, fake, fake, fake, fake, fake, fake, need - 8, nul) == -2
    assert lib.pp_field(ctypes.byref(prob), fake, fake, fake, fake, fake, nul, fake, fake, fake, 0, nul) == -2
    assert lib.pp_coeffs(ctypes.byref(prob), fake, fake, fake, fake, fake, nul, need, nul) == -1
    assert lib.pp_coeffs(ctypes.byref(prob), fake, fake, fake, fake, fake, ctypes.c_void_p((1 << 20) + 64),
                         need, nul) == -1
    # bad problem fields
    bad = P(W=-2.0)
    assert lib.pp_energy(ctypes.byref(bad), fake, fake, fake, fake, fake, fake, fake, need, nul) == -1


def test_evaluation_entry_points_validate_before_launch(lib):
    prob = P()
    st, need = ws_size(lib, prob)
    assert st == 0
    fake = ctypes.c_void_p(1 << 20)
    odd = ctypes.c_void_p((1 << 20) + 4)
    nul = None
    pf, bp = lib.pp_point_field, lib.pp_block_potential
    assert pf(None, fake, fake, fake, fake, fake, fake, fake, need, nul) == -1
    assert pf(ctypes.byref(prob), nul, fake, fake, fake, fake, fake, fake, need, nul) == -1
    assert pf(ctypes.byref(prob), fake, fake, nul, fake, fake, fake, fake, need, nul) == -1
    assert pf(ctypes.byref(prob), fake, fake, fake, odd, fake, fake, fake, need, nul) == -1
    assert pf(ctypes.byref(prob), fake, fake, fake, fake, fake, fake, fake, need - 1, nul) == -2
    assert bp(ctypes.byref(prob), fake, fake, fake, nul, fake, fake, fake, need, nul) == -1
    assert bp(ctypes.byref(prob), fake, fake, fake, fake, fake, nul, fake, need, nul) == -1
    assert bp(ctypes.byref(prob), fake, fake, fake, fake, fake, fake, fake, need - 1, nul) == -2
    # the evaluation calls regenerate the basis; the stored tables are for the gradient only
    q = P(precision=3, basis_mode=1)
    st, needq = ws_size(lib, q)
    assert st == 0
    assert pf(ctypes.byref(q), fake, fake, fake, fake, fake, fake, fake, needq, nul) == -3
    assert bp(ctypes.byref(q), fake, fake, fake, fake, fake, fake, fake, needq, nul) == -3


def test_unsupported_modes_reported(lib):
    for prec in (4, 5, 6):               # the fp8 types and the mixed split run in recompute mode only
        assert ws_size(lib, P(precision=prec))[0] == 0
        assert ws_size(lib, P(precision=prec, basis_mode=1))[0] == -3
    fake = ctypes.c_void_p(1 << 20)
    for prec in (5, 6):                  # ... and serve neither evaluation row
        q = P(precision=prec)
        st, need = ws_size(lib, q)
        assert lib.pp_point_field(ctypes.byref(q), fake, fake, fake, fake, fake, fake, fake, need, None) == -3
        assert lib.pp_block_potential(ctypes.byref(q), fake, fake, fake, fake, fake, fake, fake, need, None) == -3
    for prec in (0, 1):                  # stored tables exist for the bf16 operand types only
        st, _ = ws_size(lib, P(precision=prec, basis_mode=1))
        assert st == -3
    st, rec = ws_size(lib, P(precision=3, basis_mode=0, n=5000))
    st2, sto = ws_size(lib, P(precision=3, basis_mode=1, n=5000))
    # store adds the x3 tables: 4 bytes per (row, frequency) of each axis, rows and frequencies
    # rounded up to 256
    assert st == 0 and st2 == 0 and sto >= rec + 4 * 5120 * (256 + 256)


def test_python_binding_fails_loudly_without_gpu_tensors(lib):
    import torch
    x = torch.zeros(4, dtype=torch.float64)
    with pytest.raises(ValueError):
        pp.energy(x, x, x, x, W=1.0, H=1.0, Mu=4, Mp=4)
    with pytest.raises(ValueError):
        pp.energy(x, x, x, x, W=1.0, H=1.0, Mu=4, Mp=4, precision="fp7")


def BP(**kw):
    d = dict(W=100.0, H=50.0, n=1000, m=64, Mu=64, Mp=48)
    d.update(kw)
    return pp.PPBinProblem(d["W"], d["H"], d["n"], d["m"], d["Mu"], d["Mp"])


def bin_ws(lib, prob):
    out = ctypes.c_size_t(12345)
    st = lib.pp_bin_workspace_size(ctypes.byref(prob), ctypes.byref(out))
    return st, out.value


def test_bin_workspace_size(lib):
    st, a = bin_ws(lib, BP())
    assert st == 0 and a > 0
    st, b = bin_ws(lib, BP(m=128, Mu=128, Mp=128, n=5000))
    assert st == 0 and b > a
    assert bin_ws(lib, BP(n=0))[0] == 0
    for bad in (BP(W=0.0), BP(H=float("nan")), BP(m=0), BP(m=20000), BP(Mu=65), BP(Mp=0), BP(n=-1),
                BP(n=1 << 31)):
        assert bin_ws(lib, bad)[0] == -1
    assert lib.pp_bin_workspace_size(None, ctypes.byref(ctypes.c_size_t(0))) == -1
    assert lib.pp_bin_workspace_size(ctypes.byref(BP()), None) == -1


def test_bin_entry_points_validate_before_launch(lib):
    prob = BP()
    st, need = bin_ws(lib, prob)
    assert st == 0
    fake = ctypes.c_void_p(1 << 20)
    odd = ctypes.c_void_p((1 << 20) + 4)
    ws_odd = ctypes.c_void_p((1 << 20) + 8)
    nul = None
    bd, bc, bf = lib.pp_bin_density, lib.pp_bin_coeffs, lib.pp_bin_field
    assert bd(None, fake, fake, fake, fake, fake, fake, need, nul) == -1
    assert bd(ctypes.byref(prob), nul, fake, fake, fake, fake, fake, need, nul) == -1
    assert bd(ctypes.byref(prob), fake, fake, fake, odd, fake, fake, need, nul) == -1
    assert bd(ctypes.byref(prob), fake, fake, fake, fake, nul, fake, need, nul) == -1
    assert bd(ctypes.byref(prob), fake, fake, fake, fake, fake, fake, need - 1, nul) == -2
    assert bd(ctypes.byref(prob), fake, fake, fake, fake, fake, ws_odd, need, nul) == -1
    assert bc(ctypes.byref(prob), nul, fake, fake, need, nul) == -1
    assert bc(ctypes.byref(prob), fake, odd, fake, need, nul) == -1
    assert bc(ctypes.byref(prob), fake, fake, fake, need - 1, nul) == -2
    assert bc(ctypes.byref(BP(Mu=65)), fake, fake, fake, need, nul) == -1
    assert bf(ctypes.byref(prob), nul, fake, fake, fake, fake, need, nul) == -1
    assert bf(ctypes.byref(prob), fake, odd, fake, fake, fake, need, nul) == -1
    assert bf(ctypes.byref(prob), fake, fake, fake, fake, fake, need - 1, nul) == -2
    # nothing requested: nothing to do, after validation
    assert bf(ctypes.byref(prob), fake, nul, nul, nul, fake, need, nul) == 0
    bi = lib.pp_bin_interp
    blocks = (fake, fake, fake, fake)
    assert bi(None, *blocks, fake, nul, nul, fake, nul, nul, fake, need, nul) == -1
    # a field without its output, or an output without its field
    assert bi(ctypes.byref(prob), *blocks, fake, nul, nul, nul, nul, nul, fake, need, nul) == -1
    assert bi(ctypes.byref(prob), *blocks, nul, nul, nul, nul, fake, nul, fake, need, nul) == -1
    assert bi(ctypes.byref(prob), *blocks, nul, nul, fake, nul, nul, odd, fake, need, nul) == -1
    assert bi(ctypes.byref(prob), nul, fake, fake, fake, fake, nul, nul, fake, nul, nul, fake, need, nul) == -1
    assert bi(ctypes.byref(prob), *blocks, fake, nul, nul, fake, nul, nul, fake, need - 1, nul) == -2
    assert bi(ctypes.byref(prob), *blocks, fake, nul, nul, fake, nul, nul, ws_odd, need, nul) == -1
    # no blocks (any pointer may be NULL), or no field: nothing to do, after validation
    assert bi(ctypes.byref(BP(n=0)), nul, nul, nul, nul, fake, nul, nul, nul, nul, nul, nul, 0, nul) == 0
    assert bi(ctypes.byref(BP(n=0, m=0)), nul, nul, nul, nul, fake, nul, nul, nul, nul, nul, nul, 0, nul) == -1
    assert bi(ctypes.byref(prob), *blocks, nul, nul, nul, nul, nul, nul, fake, need, nul) == 0


# ---------------------------------------------------------------------------------------------
# Property: the host-side validation accepts exactly the problems the header documents.
# ---------------------------------------------------------------------------------------------
from hypothesis import given, settings, strategies as st  # noqa: E402

_FLOATS = st.one_of(st.floats(allow_nan=True, allow_infinity=True),
                    st.sampled_from([0.0, -0.0, -1.0, 5e-324, 1e-300, 1e300, 16384.0]))


def _documented_status(W, H, n, Mu, Mp, prec, basis):
    """The status include/pplace.h documents for a problem (its limits: n <= 2^31 - 512,
    Mu * Mp <= 2^30, and for the stored basis ceil(n / 256) * ceil(max(Mu, Mp) / 256) < 2^21)."""
    ok = lambda v: math.isfinite(v) and v > 0.0
    if (not ok(W) or not ok(H) or n < 0 or n > 2 ** 31 - 512 or not 1 <= Mu <= 65536 or not 1 <= Mp <= 65536
            or Mu * Mp > 2 ** 30 or not 0 <= prec <= 6 or basis not in (0, 1)):
        return -1
    if basis == 1 and prec not in (2, 3):
        return -3
    if basis == 1 and -(-n // 256) * -(-max(Mu, Mp) // 256) >= 2 ** 21:
        return -1
    return 0


_N = st.one_of(st.integers(-5, 2 ** 41), st.integers(2 ** 31 - 600, 2 ** 31 + 100), st.integers(0, 2 ** 27))
_M = st.one_of(st.integers(-3, 70000), st.integers(16000, 65536), st.integers(32760, 32776))


@settings(max_examples=600, deadline=None)
@given(W=_FLOATS, H=_FLOATS, n=_N, Mu=_M, Mp=_M, prec=st.integers(-2, 7), basis=st.integers(-1, 2))
def test_workspace_size_accepts_exactly_the_documented_problems(lib, W, H, n, Mu, Mp, prec, basis):
    st_, v = ws_size(lib, P(W=W, H=H, n=n, Mu=Mu, Mp=Mp, precision=prec, basis_mode=basis))
    assert st_ == _documented_status(W, H, n, Mu, Mp, prec, basis)
    if st_ == 0:
        assert v > 0 and v % 256 == 0
    else:
        assert v == 12345


@settings(max_examples=300, deadline=None)
@given(W=_FLOATS, H=_FLOATS, n=st.integers(-5, 2 ** 32), m=st.integers(-3, 20000), Mu=st.integers(-3, 20000),
       Mp=st.integers(-3, 20000))
def test_bin_workspace_size_accepts_exactly_the_documented_problems(lib, W, H, n, m, Mu, Mp):
    st_, v = bin_ws(lib, BP(W=W, H=H, n=n, m=m, Mu=Mu, Mp=Mp))
    ok = lambda x: math.isfinite(x) and x > 0.0
    valid = ok(W) and ok(H) and 0 <= n < 2 ** 31 and 1 <= m <= 16384 and 1 <= Mu <= m and 1 <= Mp <= m
    assert st_ == (0 if valid else -1)
    if valid:
        assert v > 0 and v % 256 == 0
    else:
        assert v == 12345
