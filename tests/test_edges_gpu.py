"""Degenerate and extreme cases on the GPU against the FP64 oracle, at every precision:
a single frequency (only the (0, 0) term, which the compatibility condition removes), a single
row or column of frequencies, extreme aspect ratios, tiny and region-sized blocks, blocks touching
the boundary, and a seeded sweep of random shapes (ragged sizes in every dimension)."""
import sys

import numpy as np
import pytest

import oracle
from tests import gpu_parity, parity
from workloads import Workload, make_random

torch = pytest.importorskip("torch")
pp = pytest.importorskip("paper_2307_12041_amd")

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
TOL = {"fp64": 1e-10, "fp32": 1e-5, "bf16x3": 1e-3, "bf16": 3e-2}
PRECS = ["fp64", "fp32", "bf16x3", "bf16"]


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def dev(*arrs):
    return [torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device=DEV) for a in arrs]


def rel(a, b):
    nb = np.linalg.norm(np.ravel(b))
    return np.linalg.norm(np.ravel(a) - np.ravel(b)) / (nb if nb > 0 else 1.0)


def oracle_of(wl, with_eval=True):
    """The oracle's coefficients, energy and gradients (tests/gpu_parity.py) and, with_eval, its
    block potentials and centre field of flat-spectrum coefficients (any coefficients are valid
    inputs of these linear maps; flat ones weigh every frequency tile alike)."""
    ref = gpu_parity.OracleRef(wl)
    if with_eval:
        ref.a_pt = parity.flat_point_coeffs(wl.Mu, wl.Mp, 23)
        ref.a_pot = parity.flat_potential_coeffs(wl.W, wl.H, wl.Mu, wl.Mp, 29)
        ref.N = oracle.block_potential(wl.W, wl.H, *wl.arrays(), ref.a_pot)
        po, exo, eyo = oracle.point_field(wl.W, wl.H, ref.a_pt, wl.x, wl.y)
        ref.psi, ref.xi = po, np.stack([exo, eyo], axis=1)
    return ref


def full_check(wl, prec, ref=None, with_eval=True):
    """Every metric of tests/gpu_parity.py (and, with_eval, the block potentials and the centre
    field of flat-spectrum coefficients, whole and per 256-block tile) against the oracle."""
    ref = oracle_of(wl, with_eval) if ref is None else ref
    outs = gpu_parity.run_gpu(wl, prec, ref=ref)
    errs = {k: v for k, v in gpu_parity.errors(ref, *outs).items() if not k.startswith("_")}
    if with_eval:
        x, y, w, h = dev(*wl.arrays())
        tpt, tpot = dev(ref.a_pt, ref.a_pot)
        N = pp.block_potential(x, y, w, h, tpot, W=wl.W, H=wl.H, precision=prec).cpu().numpy()
        psi, ex, ey = pp.point_field(x, y, tpt, W=wl.W, H=wl.H, precision=prec)
        xi = np.stack([ex.cpu().numpy(), ey.cpu().numpy()], axis=1)
        psi = psi.cpu().numpy()
        errs["N"], errs["N_tile"] = rel(N, ref.N), parity.row_tile_rel_max(N, ref.N)
        errs["xi"], errs["xi_tile"] = rel(xi, ref.xi), parity.row_tile_rel_max(xi, ref.xi)
        errs["psi"], errs["psi_tile"] = rel(psi, ref.psi), parity.row_tile_rel_max(psi, ref.psi)
    return errs


@pytest.mark.parametrize("prec", PRECS)
def test_single_frequency_is_all_zero(prec):
    """Mu = Mp = 1 keeps only the (0, 0) term, which the zero-mean density removes: a = E = g = 0."""
    wl = make_random(300, 50.0, 40.0, 1, 1, seed=41)
    x, y, w, h = dev(*wl.arrays())
    E, a = pp.energy(x, y, w, h, W=wl.W, H=wl.H, Mu=1, Mp=1, precision=prec)
    gx, gy = pp.field(x, y, w, h, a, W=wl.W, H=wl.H, precision=prec)
    N = pp.block_potential(x, y, w, h, a, W=wl.W, H=wl.H, precision=prec)
    assert float(a.abs().max().cpu()) == 0.0 and float(E.cpu()) == 0.0
    assert float(gx.abs().max().cpu()) == 0.0 and float(gy.abs().max().cpu()) == 0.0
    assert float(N.abs().max().cpu()) == 0.0


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("Mu,Mp", [(1, 37), (37, 1), (2, 300), (300, 2)])
def test_single_row_or_column_of_frequencies(prec, Mu, Mp):
    wl = make_random(900, 120.0, 70.0, Mu, Mp, seed=43)
    errs = full_check(wl, prec)
    say(f"[edge] Mu={Mu} Mp={Mp} {prec}: " + " ".join(f"{k}={v:.2e}" for k, v in errs.items()))
    assert max(errs.values()) <= TOL[prec], errs


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("W,H,Mu,Mp", [(100000.0, 10.0, 300, 20), (7.0, 30000.0, 24, 513)])
def test_extreme_aspect_ratios(prec, W, H, Mu, Mp):
    wl = make_random(1500, W, H, Mu, Mp, seed=47, wmax=min(8.0, W / 4), hmax=min(2.0, H / 4))
    errs = full_check(wl, prec)
    say(f"[edge] {W}x{H} M={Mu}x{Mp} {prec}: " + " ".join(f"{k}={v:.2e}" for k, v in errs.items()))
    assert max(errs.values()) <= TOL[prec], errs


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("W,H,Mu,Mp", [(1000.0, 300.0, 65536, 2), (500.0, 2000.0, 3, 65536)])
def test_maximum_frequency_count(prec, W, H, Mu, Mp):
    """The largest truncation the ABI accepts along one axis (65536 frequencies: 256 tiles of the
    bf16 kernels, 1024 K chunks of the gy contraction), 41 blocks (one whole chunk and a ragged one)."""
    wl = make_random(41, W, H, Mu, Mp, seed=59, wmax=W / 8, hmax=H / 8)
    errs = full_check(wl, prec)
    say(f"[edge] {W}x{H} M={Mu}x{Mp} {prec}: " + " ".join(f"{k}={v:.2e}" for k, v in errs.items()))
    assert max(errs.values()) <= TOL[prec], errs


@pytest.mark.parametrize("prec", PRECS)
def test_tiny_huge_and_boundary_blocks(prec):
    """Blocks of width 1e-3, blocks as large as the region, and blocks whose edge lies on the
    region boundary, mixed with ordinary ones."""
    W, H = 256.0, 128.0
    rng = np.random.default_rng(53)
    n = 600
    w = rng.uniform(1.0, 8.0, n)
    h = np.ones(n)
    w[:50] = 1e-3
    h[50:60] = 1e-3
    w[60:62] = W
    h[60:62] = H
    x = rng.uniform(0.0, W, n)
    y = rng.uniform(0.0, H, n)
    x[62:80] = w[62:80] / 2.0                   # left edge on x = 0
    x[80:100] = W - w[80:100] / 2.0             # right edge on x = W
    y[100:120] = h[100:120] / 2.0
    x[60:62] = W / 2.0
    y[60:62] = H / 2.0
    wl = Workload("edge_blocks", W, H, 160, 96, x, y, w, h, {})
    errs = full_check(wl, prec)
    say(f"[edge] tiny/huge/boundary blocks {prec}: " + " ".join(f"{k}={v:.2e}" for k, v in errs.items()))
    assert max(errs.values()) <= TOL[prec], errs


@pytest.mark.parametrize("case", range(10))
def test_random_shape_sweep(case):
    """Seeded random problems: n in [1, 4000], Mu, Mp in [1, 700], W, H in [1, 3e4]; every precision."""
    rng = np.random.default_rng(1000 + case)
    n = int(rng.integers(1, 4001))
    Mu, Mp = int(rng.integers(1, 701)), int(rng.integers(1, 701))
    W, H = float(10 ** rng.uniform(0, 4.5)), float(10 ** rng.uniform(0, 4.5))
    wl = make_random(n, W, H, Mu, Mp, seed=2000 + case, wmax=max(W / 20, 1e-2), hmax=max(H / 20, 1e-2))
    ev = case % 2 == 0
    ref = oracle_of(wl, ev)
    for prec in PRECS:
        errs = full_check(wl, prec, ref, with_eval=ev)
        say(f"[sweep {case}] n={n} M={Mu}x{Mp} {W:.3g}x{H:.3g} {prec}: "
            + " ".join(f"{k}={v:.2e}" for k, v in errs.items()))
        assert max(errs.values()) <= TOL[prec], (prec, errs)
