"""GPU parity of the FP32 path (PP_FP32) against the FP64 oracle, and the FP32 / BF16x3 / FP64
comparison on the 200,000-cell workload.

The FP32 path rounds every basis value (generated in FP64) once to FP32 (relative 2^-24) and
accumulates on v_mfma_f32_16x16x4f32 in FP32 within one K split (at most a few thousand blocks),
FP64 across splits.  With table rounding u = 6e-8 and FP32 summation of k terms bounded by
~sqrt(k) u in the norm (random rounding), the coefficient, energy and gradient errors are a few
1e-7 at k ~ 1e3; the bar is 1e-5 for every metric of tests/gpu_parity.py (whole and per-tile
errors of the flat-spectrum raw sums and of the gradients of the run's own and of flat-spectrum
coefficients)."""
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
TOL = {"fp64": 1e-10, "fp32": 1e-5, "bf16x3": 1e-3}


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def dev(*arrs):
    return [torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device=DEV) for a in arrs]


def rel(a, b):
    nb = np.linalg.norm(np.ravel(b))
    return np.linalg.norm(np.ravel(a) - np.ravel(b)) / (nb if nb > 0 else 1.0)


def run(wl, prec):
    x, y, w, h = dev(*wl.arrays())
    E, a = pp.energy(x, y, w, h, W=wl.W, H=wl.H, Mu=wl.Mu, Mp=wl.Mp, precision=prec)
    gx, gy = pp.field(x, y, w, h, a, W=wl.W, H=wl.H, precision=prec)
    torch.cuda.synchronize()
    return float(E.cpu()), a.cpu().numpy(), gx.cpu().numpy(), gy.cpu().numpy()


@pytest.mark.parametrize("n,Mu,Mp,W,H,seed", [
    (1, 5, 3, 10.0, 7.0, 0),
    (37, 24, 20, 100.0, 60.0, 1),
    (1000, 64, 64, 1024.0, 1024.0, 2),
    (3001, 300, 150, 500.0, 300.0, 3),
    (5000, 257, 513, 300.0, 900.0, 4),
    (700, 40, 600, 64.0, 800.0, 5),
])
def test_fp32_parity_shapes(n, Mu, Mp, W, H, seed):
    gpu_parity.check(make_random(n, W, H, Mu, Mp, seed=seed), "fp32", TOL["fp32"])


def test_fp32_parity_overhanging_and_macros():
    wl = make_random(800, 400.0, 300.0, 96, 80, seed=8, wmax=60.0, hmax=40.0, inside=False)
    gpu_parity.check(wl, "fp32", TOL["fp32"])


def test_precisions_cells200k_macros50_M512():
    """FP32 against the BF16 split on the coefficient contraction (and energy, gradient), with the
    FP64 path beside them; one oracle evaluation (gradients at 3000 sampled blocks) serves all three."""
    wl = make_config(2)
    say(f"[parity] {wl.name} n={wl.n} Mu={wl.Mu} Mp={wl.Mp}: fp64, fp32, bf16x3 vs oracle")
    ref = gpu_parity.OracleRef(wl, grad_sample=3000)
    for prec in ("fp64", "fp32", "bf16x3"):
        gpu_parity.check(wl, prec, TOL[prec], ref=ref)


def test_fp32_zero_blocks_and_autograd():
    say("[edge] fp32 n=0, autograd")
    x = torch.empty(0, dtype=torch.float64, device=DEV)
    E, a = pp.energy(x, x, x, x, W=10.0, H=10.0, Mu=17, Mp=9, precision="fp32")
    assert float(E.cpu()) == 0.0 and float(a.abs().max().cpu()) == 0.0
    wl = make_random(500, 60.0, 40.0, 64, 48, seed=31)
    x, y, w, h = dev(*wl.arrays())
    xr = x.clone().requires_grad_(True)
    yr = y.clone().requires_grad_(True)
    E = pp.energy_autograd(xr, yr, w, h, W=wl.W, H=wl.H, Mu=wl.Mu, Mp=wl.Mp, precision="fp32")
    E.backward()
    _, a = pp.energy(x, y, w, h, W=wl.W, H=wl.H, Mu=wl.Mu, Mp=wl.Mp, precision="fp32")
    gx, gy = pp.field(x, y, w, h, a, W=wl.W, H=wl.H, precision="fp32")
    assert torch.equal(xr.grad, gx) and torch.equal(yr.grad, gy)
