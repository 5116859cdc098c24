"""The C ABI on the GPU: argument errors are found on the host before anything is enqueued, so
device outputs keep their contents (a sentinel), and the status codes are the documented ones.
The calls go straight through ctypes to libpplace.so with real device buffers."""
import ctypes
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pp = pytest.importorskip("paper_2307_12041_amd")

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
SENT = 7.25
OK, ARG, WS, UNSUP = 0, -1, -2, -3


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def vp(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def sentinel(*shape):
    return torch.full(shape, SENT, dtype=torch.float64, device=DEV)


def untouched(*ts):
    torch.cuda.synchronize()
    return all(bool((t == SENT).all()) for t in ts)


def test_argument_errors_leave_device_outputs_untouched():
    lib = pp.load()
    st = ctypes.c_void_p(torch.cuda.current_stream(DEV).cuda_stream)
    n, Mu, Mp, W, H = 300, 40, 30, 50.0, 20.0
    rng = np.random.default_rng(3)
    x, y, w, h = (torch.as_tensor(v, device=DEV) for v in (rng.uniform(0, W, n), rng.uniform(0, H, n),
                                                            rng.uniform(0.5, 2, n), rng.uniform(0.5, 2, n)))
    blocks = [vp(t) for t in (x, y, w, h)]
    say("[abi] argument errors on the device")
    for prec in ("fp64", "bf16x3"):
        P = pp.PPProblem(W, H, n, Mu, Mp, pp.PRECISIONS[prec], 0)
        need = pp.workspace_size(W, H, n, Mu, Mp, precision=prec)
        need_fp8 = pp.workspace_size(W, H, n, Mu, Mp, precision="fp8")
        ws = torch.empty(max(need, need_fp8), dtype=torch.uint8, device=DEV)
        a, E, gx, gy, N = sentinel(Mu, Mp), sentinel(1), sentinel(n), sentinel(n), sentinel(n)
        psi, ex, ey = sentinel(n), sentinel(n), sentinel(n)
        bad = [("short workspace", P, need - 1, WS), ("W = 0", pp.PPProblem(0.0, H, n, Mu, Mp, P.precision, 0), need, ARG),
               ("H NaN", pp.PPProblem(W, float("nan"), n, Mu, Mp, P.precision, 0), need, ARG),
               ("Mu = 0", pp.PPProblem(W, H, n, 0, Mp, P.precision, 0), need, ARG),
               ("n < 0", pp.PPProblem(W, H, -1, Mu, Mp, P.precision, 0), need, ARG),
               ("FP8 evaluation rows", pp.PPProblem(W, H, n, Mu, Mp, 4, 0), need, [None, None, None, UNSUP, UNSUP]),
               ("FP8 with the workspace of another precision", pp.PPProblem(W, H, n, Mu, Mp, 4, 0), need_fp8 - 1,
                [WS, WS, WS, UNSUP, UNSUP]),
               ("unknown precision", pp.PPProblem(W, H, n, Mu, Mp, 9, 0), need, ARG)]
        if prec == "fp64":
            bad.append(("store mode in FP64", pp.PPProblem(W, H, n, Mu, Mp, 0, 1), need, UNSUP))
        for what, Q, nb, code in bad:
            codes = code if isinstance(code, list) else [code] * 5
            calls = [lambda: lib.pp_coeffs(ctypes.byref(Q), *blocks, vp(a), vp(ws), nb, st),
                     lambda: lib.pp_energy(ctypes.byref(Q), *blocks, vp(E), vp(a), vp(ws), nb, st),
                     lambda: lib.pp_field(ctypes.byref(Q), *blocks, vp(a), None, vp(gx), vp(gy), vp(ws), nb, st),
                     lambda: lib.pp_point_field(ctypes.byref(Q), vp(x), vp(y), vp(a), vp(psi), vp(ex), vp(ey), vp(ws),
                                                nb, st),
                     lambda: lib.pp_block_potential(ctypes.byref(Q), *blocks, vp(a), vp(N), vp(ws), nb, st)]
            r = [f() if c is not None else None for f, c in zip(calls, codes)]
            assert r == codes, (prec, what, r)
            assert untouched(a, E, gx, gy, N, psi, ex, ey), (prec, what)
        # a missing block array, and a misaligned output
        r1 = lib.pp_energy(ctypes.byref(P), None, *blocks[1:], vp(E), vp(a), vp(ws), need, st)
        r2 = lib.pp_field(ctypes.byref(P), *blocks, vp(a), None, ctypes.c_void_p(gx.data_ptr() + 4), vp(gy), vp(ws),
                          need, st)
        assert (r1, r2) == (ARG, ARG)
        assert untouched(a, E, gx, gy)
    # the bin scheme
    m = 32
    B = pp.PPBinProblem(W, H, n, m, m, m)
    need = pp.bin_workspace_size(W, H, n, m)
    ws = torch.empty(need, dtype=torch.uint8, device=DEV)
    P2, a2 = sentinel(m, m), sentinel(m, m)
    f1, f2, f3 = sentinel(m, m), sentinel(m, m), sentinel(m, m)
    o1, o2, o3 = sentinel(n), sentinel(n), sentinel(n)
    r = [lib.pp_bin_density(ctypes.byref(B), *blocks, vp(P2), vp(ws), need - 1, st),
         lib.pp_bin_coeffs(ctypes.byref(pp.PPBinProblem(W, H, n, m, m + 1, m)), vp(P2), vp(a2), vp(ws), need, st),
         lib.pp_bin_field(ctypes.byref(B), vp(a2), vp(f1), vp(f2), vp(f3), vp(ws), need - 1, st),
         lib.pp_bin_interp(ctypes.byref(B), *blocks, vp(f1), vp(f2), vp(f3), vp(o1), None, vp(o3), vp(ws), need, st)]
    assert r == [WS, ARG, WS, ARG], r
    assert untouched(P2, a2, f1, f2, f3, o1, o2, o3)
