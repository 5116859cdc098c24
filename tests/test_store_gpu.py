"""Store basis mode (PP_BASIS_STORE) on the GPU: the forward contracts basis tables built in HBM,
the gradient reads the tables that the forward left in the same workspace.

Bars: the FP64 oracle at the split-precision tolerance (1e-3 for bf16x3, 3e-2 for plain bf16), and
the recompute mode of the same precision (the stored tables hold the very values that the
generating forward produces, so the coefficients agree to rounding of the accumulation order,
1e-12 relative)."""
import sys

import numpy as np
import pytest

import oracle
from tests import gpu_parity
from workloads import make_config, make_random

torch = pytest.importorskip("torch")
pp = pytest.importorskip("paper_2307_12041_amd")

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
TOL = {"bf16x3": 1e-3, "bf16": 3e-2}


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def dev(*arrs):
    return [torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device=DEV) for a in arrs]


def rel(a, b):
    nb = np.linalg.norm(np.ravel(b))
    return np.linalg.norm(np.ravel(a) - np.ravel(b)) / (nb if nb > 0 else 1.0)


def run(wl, prec, basis):
    x, y, w, h = dev(*wl.arrays())
    ws = torch.empty(pp.workspace_size(wl.W, wl.H, wl.n, wl.Mu, wl.Mp, precision=prec, basis=basis),
                     dtype=torch.uint8, device=DEV)
    E, a = pp.energy(x, y, w, h, W=wl.W, H=wl.H, Mu=wl.Mu, Mp=wl.Mp, precision=prec, basis=basis, workspace=ws)
    gx, gy = pp.field(x, y, w, h, a, W=wl.W, H=wl.H, precision=prec, basis=basis, workspace=ws)
    torch.cuda.synchronize()
    return float(E.cpu()), a.cpu().numpy(), gx.cpu().numpy(), gy.cpu().numpy()


def check(wl, prec, grad_sample=None):
    """Store mode against the oracle (every metric of tests/gpu_parity.py; the flat-spectrum
    gradients read the tables that the energy call left in the workspace), and against the
    recompute mode of the same precision."""
    errs, outs = gpu_parity.check(wl, prec, TOL[prec], basis="store", grad_sample=grad_sample, label="store")
    Er, ar, _, _ = run(wl, prec, "recompute")
    esr = rel(outs[1], ar)
    say(f"   store vs recompute a={esr:.3e}")
    assert esr <= 1e-12


@pytest.mark.parametrize("prec", ["bf16x3", "bf16"])
@pytest.mark.parametrize("n,Mu,Mp,W,H,seed", [
    (1, 5, 3, 10.0, 7.0, 0),
    (37, 24, 20, 100.0, 60.0, 1),
    (1000, 64, 64, 1024.0, 1024.0, 2),
    (3001, 300, 150, 500.0, 300.0, 3),
    (5000, 257, 513, 300.0, 900.0, 4),
    (700, 40, 600, 64.0, 800.0, 5),
])
def test_store_parity_shapes(prec, n, Mu, Mp, W, H, seed):
    check(make_random(n, W, H, Mu, Mp, seed=seed), prec)


def test_store_parity_overhanging_and_macros():
    check(make_random(800, 400.0, 300.0, 96, 80, seed=8, wmax=60.0, hmax=40.0, inside=False), "bf16x3")


def test_store_parity_cells200k_macros50_M512():
    check(make_config(2), "bf16x3", grad_sample=3000)


def test_store_zero_blocks_autograd_and_workspace_contract():
    say("[store] n=0, autograd, workspace contract")
    x = torch.empty(0, dtype=torch.float64, device=DEV)
    E, a = pp.energy(x, x, x, x, W=10.0, H=10.0, Mu=17, Mp=9, precision="bf16x3", basis="store")
    assert float(E.cpu()) == 0.0 and float(a.abs().max().cpu()) == 0.0
    wl = make_random(500, 60.0, 40.0, 64, 48, seed=31)
    x, y, w, h = dev(*wl.arrays())
    xr = x.clone().requires_grad_(True)
    yr = y.clone().requires_grad_(True)
    E = pp.energy_autograd(xr, yr, w, h, W=wl.W, H=wl.H, Mu=wl.Mu, Mp=wl.Mp, precision="bf16x3", basis="store")
    E.backward()
    _, _, gx, gy = run(wl, "bf16x3", "store")
    assert np.array_equal(xr.grad.cpu().numpy(), gx) and np.array_equal(yr.grad.cpu().numpy(), gy)
    with pytest.raises(ValueError):
        pp.field(x, y, w, h, torch.zeros((64, 48), dtype=torch.float64, device=DEV), W=wl.W, H=wl.H,
                 precision="bf16x3", basis="store")
    with pytest.raises(pp.PPError):
        pp.energy(x, y, w, h, W=wl.W, H=wl.H, Mu=64, Mp=48, precision="fp64", basis="store")
