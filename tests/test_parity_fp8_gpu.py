"""GPU parity of the FP8 operand types (PP_FP8X3, PP_FP8) against the FP64 oracle.

e4m3 keeps 3 mantissa bits.  A value split into hi = e4m3(x) and lo = e4m3(x - hi) is represented to
|x - hi - lo| <= 2^-4 |lo| <= 2^-8 |x| (normal range), so one product of the x3 sum hi*hi + lo*hi +
hi*lo is off by at most (2 * 2^-8 + 2^-8 + 2^-16) |xy| ~ 1.2e-2 |xy| (the dropped lo*lo included);
plain e4m3 by (2 * 2^-4 + 2^-8) |xy| ~ 0.13 |xy|.  These per-term bounds bound the full-size
samples scaled by sum |S'T'| exactly (up to FP32 accumulation and the subnormal floor); the rounding
errors of independent terms add like random walks, so the whole-array and per-tile metrics of
tests/gpu_parity.py come out ~1e-3 (x3) and ~3e-2 (plain) and are held to 1e-2 and 0.13.
"""
import sys

import numpy as np
import pytest

import oracle
from tests import gpu_parity, parity
from workloads import make_config, make_random

torch = pytest.importorskip("torch")
pp = pytest.importorskip("paper_2307_12041_amd")

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
TOL = {"fp8x3": 1e-2, "fp8": 0.13}
SAMPLE_TOL = {"fp8x3": 1.2e-2, "fp8": 0.13}


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def dev(*arrs):
    return [torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device=DEV) for a in arrs]


SHAPES = [
    (1, 5, 3, 10.0, 7.0, 0),
    (37, 24, 20, 100.0, 60.0, 1),
    (1000, 64, 64, 1024.0, 1024.0, 2),
    (3001, 300, 150, 500.0, 300.0, 3),
    (5000, 257, 513, 300.0, 900.0, 4),
    (700, 40, 600, 64.0, 800.0, 5),
]


@pytest.mark.parametrize("prec", ["fp8x3", "fp8"])
@pytest.mark.parametrize("n,Mu,Mp,W,H,seed", SHAPES)
def test_fp8_parity_shapes(prec, n, Mu, Mp, W, H, seed):
    gpu_parity.check(make_random(n, W, H, Mu, Mp, seed=seed), prec, TOL[prec])


@pytest.mark.parametrize("prec", ["fp8x3", "fp8"])
def test_fp8_parity_overhanging_macros_and_tiny_blocks(prec):
    """Macros up to 60 x 40 overhanging the region (the size entries take their own chunk scale),
    mixed with blocks 1e-3 wide."""
    wl = make_random(800, 400.0, 300.0, 96, 80, seed=8, wmax=60.0, hmax=40.0, inside=False)
    wl.w[:40] = 1e-3
    wl.h[40:80] = 1e-3
    gpu_parity.check(wl, prec, TOL[prec])


def test_fp8_edges_zero_blocks_one_frequency_determinism_and_autograd():
    say("[fp8] n=0, Mu=Mp=1, determinism, autograd")
    x = torch.empty(0, dtype=torch.float64, device=DEV)
    for prec in ("fp8x3", "fp8"):
        E, a = pp.energy(x, x, x, x, W=10.0, H=10.0, Mu=17, Mp=9, precision=prec)
        assert float(E.cpu()) == 0.0 and float(a.abs().max().cpu()) == 0.0
    wl = make_random(300, 50.0, 40.0, 1, 1, seed=41)
    xs, ys, ws, hs = dev(*wl.arrays())
    E, a = pp.energy(xs, ys, ws, hs, W=wl.W, H=wl.H, Mu=1, Mp=1, precision="fp8x3")
    gx, gy = pp.field(xs, ys, ws, hs, a, W=wl.W, H=wl.H, precision="fp8x3")
    assert float(E.cpu()) == 0.0 and float(gx.abs().max().cpu()) == 0.0 and float(gy.abs().max().cpu()) == 0.0
    wl = make_random(20000, 700.0, 500.0, 300, 280, seed=21, wmax=8, hmax=2)
    runs = [gpu_parity.run_gpu(wl, "fp8x3") for _ in range(2)]
    for u, v in zip(*runs):
        assert np.array_equal(u, v)
    wl = make_random(500, 60.0, 40.0, 64, 48, seed=31)
    xs, ys, ws, hs = dev(*wl.arrays())
    xr, yr = xs.clone().requires_grad_(True), ys.clone().requires_grad_(True)
    E = pp.energy_autograd(xr, yr, ws, hs, W=wl.W, H=wl.H, Mu=wl.Mu, Mp=wl.Mp, precision="fp8x3")
    E.backward()
    _, a = pp.energy(xs, ys, ws, hs, W=wl.W, H=wl.H, Mu=wl.Mu, Mp=wl.Mp, precision="fp8x3")
    gx, gy = pp.field(xs, ys, ws, hs, a, W=wl.W, H=wl.H, precision="fp8x3")
    assert torch.equal(xr.grad, gx) and torch.equal(yr.grad, gy)
    with pytest.raises(pp.PPError):
        pp.point_field(xs, ys, a, W=wl.W, H=wl.H, precision="fp8x3")


@pytest.mark.parametrize("prec", ["fp8x3", "fp8"])
def test_fp8_bench_workload_cells2m_macros500_M2048(prec):
    """At 2,000,500 blocks and 2048 x 2048 frequencies: three sampled coefficients in every 256 x 256
    tile against the oracle, each scaled by f_up sum_i |S'_iu T'_ip| (bounded by the per-term error),
    and the gradients of flat-spectrum coefficients at 64 sampled blocks (the 16 largest macros
    among them)."""
    wl = make_config(4)
    say(f"[fp8 workload] {wl.name} n={wl.n} M={wl.Mu}x{wl.Mp} prec={prec}")
    x, y, w, h = (torch.as_tensor(v, device=DEV) for v in wl.arrays())
    ws = torch.empty(pp.workspace_size(wl.W, wl.H, wl.n, wl.Mu, wl.Mp, precision=prec), dtype=torch.uint8,
                     device=DEV)
    E, a = pp.energy(x, y, w, h, W=wl.W, H=wl.H, Mu=wl.Mu, Mp=wl.Mp, precision=prec, workspace=ws)
    torch.cuda.synchronize()
    an = a.cpu().numpy()
    us, ps = parity.samples_per_tile(wl.Mu, wl.Mp, 3, 4)
    ao, _, Rabs = oracle.coeffs_sampled_full(wl.W, wl.H, *wl.arrays(), us, ps)
    f = oracle.coef_factors(wl.W, wl.H, wl.Mu, wl.Mp)[us, ps]
    errs = parity.scaled_sample_errors(an[us, ps], ao, f, Rabs)
    tiles = parity.tile_max_of_samples(errs, us, ps)
    worst = max(tiles.values())
    say(f"   {len(us)} sampled coefficients in {len(tiles)} tiles: worst scaled error {worst:.2e}, "
        f"median {np.median(errs):.2e}; relative norm {parity.rel(an[us, ps], ao):.2e}")
    assert worst <= SAMPLE_TOL[prec]
    idx = np.unique(np.concatenate([np.random.default_rng(44).choice(wl.n, 48, replace=False),
                                    np.argsort(wl.w * wl.h)[-16:]]))
    a_x, a_y = parity.flat_field_coeffs(wl.W, wl.H, wl.Mu, wl.Mp, 44)
    gxo, _ = oracle.grad_sampled(wl.W, wl.H, *wl.arrays(), a_x, idx)
    _, gyo = oracle.grad_sampled(wl.W, wl.H, *wl.arrays(), a_y, idx)
    gx, _ = pp.field(x, y, w, h, torch.as_tensor(a_x, device=DEV), W=wl.W, H=wl.H, precision=prec, workspace=ws)
    _, gy = pp.field(x, y, w, h, torch.as_tensor(a_y, device=DEV), W=wl.W, H=wl.H, precision=prec, workspace=ws)
    torch.cuda.synchronize()
    eg = (parity.rel(gx.cpu().numpy()[idx], gxo), parity.rel(gy.cpu().numpy()[idx], gyo))
    say(f"   gradients of flat-spectrum coefficients at {len(idx)} blocks: gx {eg[0]:.2e} gy {eg[1]:.2e}")
    assert max(eg) <= TOL[prec]
