"""The large workloads at full size, on the GPU.

* 2,000,000 cells + 500 macros in 16384 x 16384, M = 2048 x 2048, in the benchmark's launch
  configuration (BF16X3, basis regenerated on chip, one caller workspace for energy and gradient):
  three sampled coefficients in every 256 x 256 output tile against the oracle (each a direct sum
  over all blocks, compared on its own, scaled by f_up sum_i |S'_iu T'_ip|); the gradients of
  flat-spectrum coefficients (every frequency tile weighs alike) at sampled blocks (the largest
  macros among them) against the oracle, in BF16X3 and FP64; and E = 1/2 sum_up a_up^2 / s_up over
  the GPU's own coefficients.
* 1,000,000 cells in 16 Gaussian clusters (sigma 800) in 16384 x 16384, M = 1024 x 1024: forces from
  the differentiable energy (torch.autograd through the hand-written backward) against central
  differences with h = 1e-3 on 100 seeded random blocks, and three sampled FP64 coefficients in
  every tile against the oracle.
* 10,000,000 cells (70% in 64 clusters, 30% uniform) in 32768 x 16384, M = 4096 x 2048: ten
  evaluations with N(0, 1) jittered positions; sampled coefficients in every tile against the
  oracle at the first and last iteration, and at the last the central-difference check of the
  forces and the flat-spectrum gradients against the oracle.

Expected values come from the oracle and seeded inputs only.  The central differences are a
consistency property of the GPU's own outputs (its forces are the derivative of its energy): they
use the exact rank-one energy change of one moved block (tests/fd_rank1.py, pinned against the
oracle's gradient on the CPU) with the FP64 GPU coefficients of the same blocks, so they hold at any
size; the oracle comparisons of the gradient use flat-spectrum coefficients instead.
"""
import sys

import numpy as np
import pytest

import oracle
from tests import parity
from tests.fd_rank1 import _scale, central_difference
from workloads import jitter, make_config

torch = pytest.importorskip("torch")
pp = pytest.importorskip("paper_2307_12041_amd")

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def rel(a, b):
    nb = np.linalg.norm(np.ravel(b))
    return np.linalg.norm(np.ravel(a) - np.ravel(b)) / (nb if nb > 0 else 1.0)


SAMPLE_TOL = {"bf16x3": 1e-5, "fp64": 1e-13}   # per-sample errors scaled by f_up sum_i |S'_iu T'_ip|


def sampled_coeff_check(wl, a, prec, per_tile, seed, tag=""):
    """Sampled coefficients, `per_tile` of them in every 256 x 256 output tile of the bf16
    contractions, each a direct oracle sum over all blocks and compared on its own: |a - a*| scaled
    by f_up sum_i |S'_iu T'_ip| (the magnitude that bounds the rounding of its sum; a zeroed tile is
    ~n^-1/2 off, see tests/test_parity_metrics.py), and the worst such error of every tile."""
    us, ps = parity.samples_per_tile(wl.Mu, wl.Mp, per_tile, seed)
    ao, _, Rabs = oracle.coeffs_sampled_full(wl.W, wl.H, *wl.arrays(), us, ps)
    f = oracle.coef_factors(wl.W, wl.H, wl.Mu, wl.Mp)[us, ps]
    errs = parity.scaled_sample_errors(a[us, ps], ao, f, Rabs)
    tiles = parity.tile_max_of_samples(errs, us, ps)
    worst = max(tiles, key=tiles.get)
    say(f"   {tag}{len(us)} sampled coefficients in {len(tiles)} tiles vs oracle: worst scaled error "
        f"{tiles[worst]:.2e} (tile {worst}), median {np.median(errs):.2e}; relative norm {rel(a[us, ps], ao):.2e}")
    assert tiles[worst] <= SAMPLE_TOL[prec], (prec, worst, tiles[worst])
    return tiles


def sampled_flat_gradient_check(wl, x, y, w, h, idx, prec, tol, seed, ws=None):
    """Gradients of flat-spectrum coefficients (the gx operand a / vt and the gy operand a / wt
    ~N(0, 1) over the whole frequency plane) at the sampled blocks against the oracle: the relative
    norm and the largest block error over the rms of the oracle's values."""
    a_x, a_y = parity.flat_field_coeffs(wl.W, wl.H, wl.Mu, wl.Mp, seed)
    gxo, _ = oracle.grad_sampled(wl.W, wl.H, *wl.arrays(), a_x, idx)
    _, gyo = oracle.grad_sampled(wl.W, wl.H, *wl.arrays(), a_y, idx)
    gx, _ = pp.field(x, y, w, h, torch.as_tensor(a_x, device=DEV), W=wl.W, H=wl.H, precision=prec, workspace=ws)
    _, gy = pp.field(x, y, w, h, torch.as_tensor(a_y, device=DEV), W=wl.W, H=wl.H, precision=prec, workspace=ws)
    torch.cuda.synchronize()
    out = {}
    for name, g, go in (("gx", gx.cpu().numpy()[idx], gxo), ("gy", gy.cpu().numpy()[idx], gyo)):
        rms = float(np.sqrt(np.mean(go * go)))
        out[name] = rel(g, go)
        out[name + "_maxblock"] = float(np.max(np.abs(g - go))) / rms
    say(f"   {prec} gradients of flat-spectrum coefficients at {len(idx)} blocks vs oracle: "
        + " ".join(f"{k}={v:.2e}" for k, v in out.items()))
    assert max(out.values()) <= tol, (prec, out)
    return out


def test_bench_workload_cells2m_macros500_M2048():
    wl = make_config(4)
    say(f"[workload] {wl.name} n={wl.n} Mu={wl.Mu} Mp={wl.Mp}, bf16x3 recompute")
    x, y, w, h = (torch.as_tensor(v, device=DEV) for v in wl.arrays())
    need = pp.workspace_size(wl.W, wl.H, wl.n, wl.Mu, wl.Mp, precision="bf16x3")
    ws = torch.empty(need, dtype=torch.uint8, device=DEV)
    E, a = pp.energy(x, y, w, h, W=wl.W, H=wl.H, Mu=wl.Mu, Mp=wl.Mp, precision="bf16x3", workspace=ws)
    gx, gy = pp.field(x, y, w, h, a, W=wl.W, H=wl.H, precision="bf16x3", workspace=ws)
    torch.cuda.synchronize()
    an = a.cpu().numpy()
    assert bool(torch.isfinite(gx).all()) and bool(torch.isfinite(gy).all())
    # coefficients: three samples in every 256 x 256 tile, each a direct oracle sum over all blocks
    sampled_coeff_check(wl, an, "bf16x3", 3, 4)
    # energy over the GPU's own coefficients: E = 1/2 sum a^2 / s (a = s A)
    s = _scale(wl.W, wl.H, wl.Mu, wl.Mp)
    nz = s > 0
    Ev = float(E.cpu())
    eE = abs(0.5 * np.sum(an[nz] ** 2 / s[nz]) - Ev) / Ev
    say(f"   |E - 1/2 sum a^2/s| / E = {eE:.2e}")
    assert eE < 1e-6
    # gradients of flat-spectrum coefficients at sampled blocks, the 16 largest macros among them
    idx = np.unique(np.concatenate([np.random.default_rng(44).choice(wl.n, 48, replace=False),
                                    np.argsort(wl.w * wl.h)[-16:]]))
    for prec, tol in (("bf16x3", 1e-3), ("fp64", 1e-10)):
        sampled_flat_gradient_check(wl, x, y, w, h, idx, prec, tol, 44, ws=ws if prec == "bf16x3" else None)


def test_clusters_1m_autograd_forces_vs_central_differences():
    wl = make_config(3)
    say(f"[workload] {wl.name} n={wl.n} Mu={wl.Mu} Mp={wl.Mp}")
    x, y, w, h = (torch.as_tensor(v, device=DEV) for v in wl.arrays())
    xr = x.clone().requires_grad_(True)
    yr = y.clone().requires_grad_(True)
    E = pp.energy_autograd(xr, yr, w, h, W=wl.W, H=wl.H, Mu=wl.Mu, Mp=wl.Mp, precision="bf16x3")
    E.backward()
    E64, a64 = pp.energy(x, y, w, h, W=wl.W, H=wl.H, Mu=wl.Mu, Mp=wl.Mp, precision="fp64")
    gx64, gy64 = pp.field(x, y, w, h, a64, W=wl.W, H=wl.H, precision="fp64")
    torch.cuda.synchronize()
    a64n = a64.cpu().numpy()
    idx = np.sort(np.random.default_rng(3).choice(wl.n, 100, replace=False))
    fx, fy = central_difference(wl.W, wl.H, *wl.arrays(), a64n, idx, 1e-3)
    fd = np.concatenate([fx, fy])
    g64 = np.concatenate([gx64.cpu().numpy()[idx], gy64.cpu().numpy()[idx]])
    gbf = np.concatenate([xr.grad.cpu().numpy()[idx], yr.grad.cpu().numpy()[idx]])
    e64, ebf = rel(g64, fd), rel(gbf, fd)
    say(f"   forces vs central differences: fp64 {e64:.2e}, bf16x3 autograd {ebf:.2e}")
    assert e64 < 1e-7
    assert ebf < 1e-3
    eE = abs(float(E.detach().cpu()) - float(E64.cpu())) / abs(float(E64.cpu()))
    assert eE < 1e-3
    say(f"   energy bf16x3 vs fp64 {eE:.2e}")
    sampled_coeff_check(wl, a64n, "fp64", 3, 5, tag="fp64: ")


def test_clusters_10m_jittered_iterations():
    base = make_config(5)
    say(f"[workload] {base.name} n={base.n} Mu={base.Mu} Mp={base.Mp}, 10 jittered iterations")
    w = torch.as_tensor(base.w, device=DEV)
    h = torch.as_tensor(base.h, device=DEV)
    need = pp.workspace_size(base.W, base.H, base.n, base.Mu, base.Mp, precision="bf16x3")
    ws = torch.empty(need, dtype=torch.uint8, device=DEV)
    energies = []
    for it in range(10):
        wl = jitter(base, it)
        x = torch.as_tensor(wl.x, device=DEV)
        y = torch.as_tensor(wl.y, device=DEV)
        E, a = pp.energy(x, y, w, h, W=wl.W, H=wl.H, Mu=wl.Mu, Mp=wl.Mp, precision="bf16x3", workspace=ws)
        gx, gy = pp.field(x, y, w, h, a, W=wl.W, H=wl.H, precision="bf16x3", workspace=ws)
        torch.cuda.synchronize()
        Ev = float(E.cpu())
        energies.append(Ev)
        assert np.isfinite(Ev) and Ev > 0
        assert bool(torch.isfinite(gx).all()) and bool(torch.isfinite(gy).all())
        say(f"   iteration {it}: E = {Ev:.10e}")
        if it in (0, 9):
            # one sample in every 256 x 256 tile at the first iteration, two at the last
            sampled_coeff_check(wl, a.cpu().numpy(), "bf16x3", 1 if it == 0 else 2, 11 + it)
        if it == 9:
            idx = np.sort(np.random.default_rng(9).choice(wl.n, 12, replace=False))
            fx, fy = central_difference(wl.W, wl.H, *wl.arrays(), a.cpu().numpy(), idx, 1e-3)
            g = np.concatenate([gx.cpu().numpy()[idx], gy.cpu().numpy()[idx]])
            eg = rel(g, np.concatenate([fx, fy]))
            say(f"   forces vs central differences of the same coefficients: {eg:.2e}")
            assert eg < 1e-3
            sampled_flat_gradient_check(wl, x, y, w, h, idx, "bf16x3", 1e-3, 55, ws=ws)
    # jitter of sigma = 1 on 32768 x 16384 barely moves the energy
    assert max(energies) / min(energies) < 1.01
