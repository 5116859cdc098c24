"""pp_energy_static, the allocation-free variant of pp_energy, through the C ABI on the GPU.

It runs the same kernels on the same launch plan as pp_energy, with its workspace in the library's
per-device static array instead of a caller workspace, so its energy and coefficients must equal
pp_energy's bit for bit.  Two calls in a row, the second with a smaller problem, check that what the
first call left in the shared array does not leak into the second; every precision is covered.
Problems beyond PP_STATIC_SCRATCH_BYTES and the stored basis are rejected on the host."""
import ctypes
import sys

import numpy as np
import pytest

from workloads import make_random

torch = pytest.importorskip("torch")
pp = pytest.importorskip("paper_2307_12041_amd")

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
PP_STATIC_SCRATCH_BYTES = 128 << 20


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def _args(wl, prec):
    x, y, w, h = (torch.as_tensor(np.ascontiguousarray(v), device=DEV) for v in wl.arrays())
    P = pp.PPProblem(wl.W, wl.H, wl.n, wl.Mu, wl.Mp, pp.PRECISIONS[prec], 0)
    return P, x, y, w, h


def static_call(wl, prec):
    lib = pp.load()
    P, x, y, w, h = _args(wl, prec)
    E = torch.full((), float("nan"), dtype=torch.float64, device=DEV)
    a = torch.full((wl.Mu, wl.Mp), float("nan"), dtype=torch.float64, device=DEV)
    st = lib.pp_energy_static(ctypes.byref(P), *(ctypes.c_void_p(t.data_ptr()) for t in (x, y, w, h, E, a)),
                              ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == 0, pp.load().pp_strerror(st)
    torch.cuda.synchronize()
    return float(E.cpu()), a.cpu().numpy()


def workspace_call(wl, prec):
    P, x, y, w, h = _args(wl, prec)
    E, a = pp.energy(x, y, w, h, W=wl.W, H=wl.H, Mu=wl.Mu, Mp=wl.Mp, precision=prec)
    torch.cuda.synchronize()
    return float(E.cpu()), a.cpu().numpy()


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3", "bf16"])
def test_static_energy_equals_workspace_energy_twice(prec):
    big = make_random(3001, 500.0, 300.0, 300, 150, seed=3)
    small = make_random(700, 64.0, 80.0, 40, 60, seed=5)
    for wl in (big, small):
        need = pp.workspace_size(wl.W, wl.H, wl.n, wl.Mu, wl.Mp, precision=prec)
        assert need <= PP_STATIC_SCRATCH_BYTES
        say(f"[static] {prec} n={wl.n} M={wl.Mu}x{wl.Mp} workspace {need / 2**20:.1f} MiB")
        Es, as_ = static_call(wl, prec)
        Ew, aw = workspace_call(wl, prec)
        assert np.isfinite(Es) and Es == Ew, (Es, Ew)
        assert np.array_equal(as_, aw)


def test_static_energy_rejects_what_it_cannot_hold():
    lib = pp.load()
    fake = ctypes.c_void_p(1 << 20)      # never dereferenced: both calls fail on the host
    too_big = pp.PPProblem(16384.0, 16384.0, 200050, 512, 512, pp.PRECISIONS["bf16x3"], 0)
    assert lib.pp_energy_static(ctypes.byref(too_big), fake, fake, fake, fake, fake, fake, None) == -5
    store = pp.PPProblem(500.0, 300.0, 3001, 300, 150, pp.PRECISIONS["bf16x3"], 1)
    assert lib.pp_energy_static(ctypes.byref(store), fake, fake, fake, fake, fake, fake, None) == -3
    assert b"static scratch" in lib.pp_strerror(-5)
