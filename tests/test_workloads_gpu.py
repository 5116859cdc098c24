"""The large workloads at full size, on the GPU.

* 2,000,000 cells + 500 macros in 16384 x 16384, M = 2048 x 2048, in the benchmark's launch
  configuration (BF16X3, basis regenerated on chip, one caller workspace for energy and gradient):
  sampled coefficients against the oracle (each a direct sum over all blocks); the gradient of
  seeded synthetic coefficients at sampled blocks (the largest macros among them) against the
  oracle, in BF16X3 and FP64; and E = 1/2 sum_up a_up^2 / s_up over the GPU's own coefficients.
* 1,000,000 cells in 16 Gaussian clusters (sigma 800) in 16384 x 16384, M = 1024 x 1024: forces from
  the differentiable energy (torch.autograd through the hand-written backward) against central
  differences with h = 1e-3 on 100 seeded random blocks, and sampled coefficients against the oracle.
* 10,000,000 cells (70% in 64 clusters, 30% uniform) in 32768 x 16384, M = 4096 x 2048: ten
  evaluations with N(0, 1) jittered positions; sampled coefficients against the oracle at the first
  and last iteration and the central-difference check of the forces at the last.

Expected values come from the oracle and seeded inputs only.  The central differences are a
consistency property of the GPU's own outputs (its forces are the derivative of its energy): they
use the exact rank-one energy change of one moved block (tests/fd_rank1.py, pinned against the
oracle's gradient on the CPU) with the FP64 GPU coefficients of the same blocks, so they hold at any
size; the oracle comparisons of the gradient use seeded coefficients instead.
"""
import sys

import numpy as np
import pytest

import oracle
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


def sample_uv(Mu, Mp, k, seed):
    rng = np.random.default_rng(seed)
    us = np.concatenate([[1, 0, 1, 2], rng.integers(0, Mu, k - 4)])
    ps = np.concatenate([[0, 1, 1, 3], rng.integers(0, Mp, k - 4)])
    return us, ps


def seeded_coeffs(Mu, Mp, seed):
    """Synthetic coefficients with the spectrum of real ones (falling like 1/(u^2 + p^2)), a_00 = 0."""
    rng = np.random.default_rng(seed)
    u, p = np.meshgrid(np.arange(Mu), np.arange(Mp), indexing="ij")
    a = rng.normal(size=(Mu, Mp)) / (1.0 + u * u + p * p)
    a[0, 0] = 0.0
    return a


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
    # coefficients: sampled (u, p), each a direct oracle sum over all 2,000,500 blocks
    us, ps = sample_uv(wl.Mu, wl.Mp, 32, 4)
    us[-2:], ps[-2:] = (wl.Mu - 1, 0), (0, wl.Mp - 1)
    ao, _ = oracle.coeffs_sampled(wl.W, wl.H, *wl.arrays(), us, ps)
    ea = rel(an[us, ps], ao)
    # energy over the GPU's own coefficients: E = 1/2 sum a^2 / s (a = s A)
    s = _scale(wl.W, wl.H, wl.Mu, wl.Mp)
    nz = s > 0
    Ev = float(E.cpu())
    eE = abs(0.5 * np.sum(an[nz] ** 2 / s[nz]) - Ev) / Ev
    say(f"   sampled coefficients vs oracle {ea:.2e}; |E - 1/2 sum a^2/s| / E = {eE:.2e}")
    assert ea < 1e-3 and eE < 1e-6
    # gradient of seeded coefficients at sampled blocks, the 16 largest macros among them
    a_syn = seeded_coeffs(wl.Mu, wl.Mp, 44)
    a_dev = torch.as_tensor(a_syn, device=DEV)
    idx = np.unique(np.concatenate([np.random.default_rng(44).choice(wl.n, 48, replace=False),
                                    np.argsort(wl.w * wl.h)[-16:]]))
    gxo, gyo = oracle.grad_sampled(wl.W, wl.H, *wl.arrays(), a_syn, idx)
    go = np.concatenate([gxo, gyo])
    for prec, tol in (("bf16x3", 1e-3), ("fp64", 1e-10)):
        gxs, gys = pp.field(x, y, w, h, a_dev, W=wl.W, H=wl.H, precision=prec, workspace=ws if prec == "bf16x3"
                            else None)
        torch.cuda.synchronize()
        eg = rel(np.concatenate([gxs.cpu().numpy()[idx], gys.cpu().numpy()[idx]]), go)
        say(f"   {prec} gradient of seeded coefficients at {len(idx)} blocks vs oracle {eg:.2e}")
        assert eg < tol, (prec, eg)


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
    us, ps = sample_uv(wl.Mu, wl.Mp, 24, 5)
    ao, _ = oracle.coeffs_sampled(wl.W, wl.H, *wl.arrays(), us, ps)
    ea64 = rel(a64n[us, ps], ao)
    say(f"   sampled coefficients vs oracle: fp64 {ea64:.2e}, energy bf16x3 vs fp64 {eE:.2e}")
    assert ea64 < 1e-10


def test_clusters_10m_jittered_iterations():
    base = make_config(5)
    say(f"[workload] {base.name} n={base.n} Mu={base.Mu} Mp={base.Mp}, 10 jittered iterations")
    w = torch.as_tensor(base.w, device=DEV)
    h = torch.as_tensor(base.h, device=DEV)
    need = pp.workspace_size(base.W, base.H, base.n, base.Mu, base.Mp, precision="bf16x3")
    ws = torch.empty(need, dtype=torch.uint8, device=DEV)
    us, ps = sample_uv(base.Mu, base.Mp, 8, 11)
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
            an = a.cpu().numpy()
            ao, _ = oracle.coeffs_sampled(wl.W, wl.H, *wl.arrays(), us, ps)
            ea = rel(an[us, ps], ao)
            say(f"   sampled coefficients vs oracle: {ea:.2e}")
            assert ea < 1e-3
        if it == 9:
            idx = np.sort(np.random.default_rng(9).choice(wl.n, 12, replace=False))
            fx, fy = central_difference(wl.W, wl.H, *wl.arrays(), a.cpu().numpy(), idx, 1e-3)
            g = np.concatenate([gx.cpu().numpy()[idx], gy.cpu().numpy()[idx]])
            eg = rel(g, np.concatenate([fx, fy]))
            say(f"   forces vs central differences of the same coefficients: {eg:.2e}")
            assert eg < 1e-3
            a_syn = seeded_coeffs(wl.Mu, wl.Mp, 55)
            gxs, gys = pp.field(x, y, w, h, torch.as_tensor(a_syn, device=DEV), W=wl.W, H=wl.H,
                                precision="bf16x3", workspace=ws)
            torch.cuda.synchronize()
            gxo, gyo = oracle.grad_sampled(wl.W, wl.H, *wl.arrays(), a_syn, idx)
            eg = rel(np.concatenate([gxs.cpu().numpy()[idx], gys.cpu().numpy()[idx]]), np.concatenate([gxo, gyo]))
            say(f"   gradient of seeded coefficients vs oracle: {eg:.2e}")
            assert eg < 1e-3
    # jitter of sigma = 1 on 32768 x 16384 barely moves the energy
    assert max(energies) / min(energies) < 1.01
