"""The bin scheme of Sec. III-D (the comparison path) on the GPU against the FP64 oracle:
densities, coefficients, bin-centre potential and field, and the block values weighted back
from the bins.

Bars: FP64 throughout, 1e-12 relative to the largest magnitude of each output (the densities are
FP64 atomic sums, so their last bits depend on the order of arrival; the transforms are FP64
GEMMs whose sums run in another order than the oracle's long-double ones).  At the full
2048-bin grid of the 2M-block workload the checks are the total-area invariant of the densities
and sampled bins and coefficients that the oracle computes one by one."""
import sys

import numpy as np
import pytest

import oracle
from workloads import make_config, make_random

torch = pytest.importorskip("torch")
pp = pytest.importorskip("paper_2307_12041_amd")

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
TOL = 1e-12


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def dev(*arrs):
    return [torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device=DEV) for a in arrs]


def relmax(got, want):
    s = np.abs(want).max()
    return np.abs(got - want).max() / (s if s > 0 else 1.0)


def mixed_blocks(n, W, H, seed, n_macros=12):
    """Cells of all sizes (some overhanging the region) plus macros that cover many bins."""
    wl = make_random(n, W, H, 8, 8, seed=seed, wmax=W / 20, hmax=H / 20, inside=False)
    rng = np.random.default_rng(seed + 100)
    mx, my = rng.uniform(0, W, n_macros), rng.uniform(0, H, n_macros)
    mw, mh = rng.uniform(W / 10, W / 2, n_macros), rng.uniform(H / 10, H / 2, n_macros)
    return (np.concatenate([wl.x, mx]), np.concatenate([wl.y, my]), np.concatenate([wl.w, mw]),
            np.concatenate([wl.h, mh]))


@pytest.mark.parametrize("m", [1, 7, 64, 200])
def test_bin_density_parity(m):
    W, H = 300.0, 170.0
    x, y, w, h = mixed_blocks(3000, W, H, seed=m)
    say(f"[bins] density m={m} n={len(x)}")
    P = pp.bin_density(*dev(x, y, w, h), W=W, H=H, m=m).cpu().numpy()
    ref = oracle.bin_density(W, H, x, y, w, h, m)
    assert relmax(P, ref) <= TOL


def test_bin_density_no_blocks_and_outside_blocks():
    W, H, m = 10.0, 10.0, 16
    e = torch.empty(0, dtype=torch.float64, device=DEV)
    assert float(pp.bin_density(e, e, e, e, W=W, H=H, m=m).abs().max().cpu()) == 0.0
    # entirely outside the region: in no bin
    x, y, w, h = dev([-5.0, 15.0, 5.0], [5.0, 5.0, 12.0], [2.0, 2.0, 2.0], [2.0, 2.0, 1.0])
    assert float(pp.bin_density(x, y, w, h, W=W, H=H, m=m).abs().max().cpu()) == 0.0


@pytest.mark.parametrize("m,Mu,Mp", [(1, 1, 1), (8, 8, 8), (33, 33, 20), (64, 64, 64), (100, 70, 100), (130, 130, 3)])
def test_bin_coeffs_parity(m, Mu, Mp):
    W, H = 40.0, 25.0
    P = np.random.default_rng(m * 7 + Mp).uniform(0.0, 1.5, (m, m))
    say(f"[bins] coeffs m={m} Mu={Mu} Mp={Mp}")
    a = pp.bin_coeffs(*dev(P), W=W, H=H, Mu=Mu, Mp=Mp).cpu().numpy()
    ref = oracle.bin_coeffs(W, H, P, Mu, Mp)
    assert a[0, 0] == 0.0
    if m > 1:
        assert relmax(a, ref) <= TOL


@pytest.mark.parametrize("m,Mu,Mp", [(8, 8, 8), (33, 20, 33), (70, 70, 41)])
def test_bin_field_parity(m, Mu, Mp):
    W, H = 13.0, 29.0
    a = np.random.default_rng(m + Mu).normal(size=(Mu, Mp))
    say(f"[bins] field m={m} Mu={Mu} Mp={Mp}")
    psi, xix, xiy = (t.cpu().numpy() for t in pp.bin_field(*dev(a), W=W, H=H, m=m))
    rp, rx, ry = oracle.bin_field(W, H, m, a)
    assert relmax(psi, rp) <= TOL and relmax(xix, rx) <= TOL and relmax(xiy, ry) <= TOL
    # outputs not asked for are not computed; the others are unchanged
    psi2, n1, n2 = pp.bin_field(*dev(a), W=W, H=H, m=m, want=("psi",))
    assert n1 is None and n2 is None and np.array_equal(psi2.cpu().numpy(), psi)
    _, _, y2 = pp.bin_field(*dev(a), W=W, H=H, m=m, want=("xiy",))
    assert np.array_equal(y2.cpu().numpy(), xiy)


def test_bin_pipeline_matches_oracle_pipeline():
    W, H, m = 120.0, 80.0, 48
    x, y, w, h = mixed_blocks(2000, W, H, seed=5, n_macros=4)
    say(f"[bins] pipeline m={m}")
    ws = torch.empty(pp.bin_workspace_size(W, H, len(x), m), dtype=torch.uint8, device=DEV)
    P = pp.bin_density(*dev(x, y, w, h), W=W, H=H, m=m, workspace=ws)
    a = pp.bin_coeffs(P, W=W, H=H, Mu=m, Mp=m, workspace=ws)
    psi, xix, xiy = pp.bin_field(a, W=W, H=H, m=m, workspace=ws)
    Po = oracle.bin_density(W, H, x, y, w, h, m)
    ao = oracle.bin_coeffs(W, H, Po, m, m)
    po, xo, yo = oracle.bin_field(W, H, m, ao)
    assert relmax(a.cpu().numpy(), ao) <= TOL
    assert relmax(psi.cpu().numpy(), po) <= TOL
    assert relmax(xix.cpu().numpy(), xo) <= TOL and relmax(xiy.cpu().numpy(), yo) <= TOL
    N, gx, gy = pp.bin_interp(*dev(x, y, w, h), psi, xix, xiy, W=W, H=H, workspace=ws)
    No, gxo, gyo = oracle.bin_interp(W, H, x, y, w, h, m, po, xo, yo)
    assert relmax(N.cpu().numpy(), No) <= TOL
    assert relmax(gx.cpu().numpy(), gxo) <= TOL and relmax(gy.cpu().numpy(), gyo) <= TOL


@pytest.mark.parametrize("m", [1, 7, 64, 200])
def test_bin_interp_parity(m):
    W, H = 300.0, 170.0
    x, y, w, h = mixed_blocks(3000, W, H, seed=40 + m)
    rng = np.random.default_rng(m)
    fields = [rng.normal(size=(m, m)) for _ in range(3)]
    say(f"[bins] interp m={m} n={len(x)}")
    got = pp.bin_interp(*dev(x, y, w, h), *dev(*fields), W=W, H=H)
    ref = oracle.bin_interp(W, H, x, y, w, h, m, *fields)
    for g, r in zip(got, ref):
        assert relmax(g.cpu().numpy(), r) <= TOL


def test_bin_interp_pairs_and_determinism():
    W, H, m = 90.0, 60.0, 40
    x, y, w, h = mixed_blocks(5000, W, H, seed=3, n_macros=30)
    rng = np.random.default_rng(9)
    psi, xix, xiy = dev(*[rng.normal(size=(m, m)) for _ in range(3)])
    t = dev(x, y, w, h)
    say("[bins] interp pairs")
    full = [o.cpu().numpy() for o in pp.bin_interp(*t, psi, xix, xiy, W=W, H=H)]
    again = [o.cpu().numpy() for o in pp.bin_interp(*t, psi, xix, xiy, W=W, H=H)]
    # per-block sums in a fixed order (one workgroup with a fixed-order reduction for big blocks)
    assert all(np.array_equal(a, b) for a, b in zip(full, again))
    N, n1, n2 = pp.bin_interp(*t, psi, W=W, H=H)
    assert n1 is None and n2 is None and np.array_equal(N.cpu().numpy(), full[0])
    n0, n1, gy = pp.bin_interp(*t, xiy=xiy, W=W, H=H)
    assert n0 is None and n1 is None and np.array_equal(gy.cpu().numpy(), full[2])
    e = torch.empty(0, dtype=torch.float64, device=DEV)
    N0, _, _ = pp.bin_interp(e, e, e, e, psi, W=W, H=H)
    assert N0.numel() == 0


def test_bin_full_grid_2m_blocks_sampled():
    wl = make_config(4)
    m = wl.Mu
    say(f"[bins] full grid m={m} n={wl.n}")
    x, y, w, h = dev(*wl.arrays())
    P = pp.bin_density(x, y, w, h, W=wl.W, H=wl.H, m=m)
    a = pp.bin_coeffs(P, W=wl.W, H=wl.H, Mu=m, Mp=m)
    psi, xix, xiy = pp.bin_field(a, W=wl.W, H=wl.H, m=m)
    torch.cuda.synchronize()
    Ph, ah = P.cpu().numpy(), a.cpu().numpy()
    # total area inside the region
    inside = (np.clip(np.minimum(wl.x + wl.w / 2, wl.W) - np.maximum(wl.x - wl.w / 2, 0), 0, None)
              * np.clip(np.minimum(wl.y + wl.h / 2, wl.H) - np.maximum(wl.y - wl.h / 2, 0), 0, None))
    assert Ph.sum() * (wl.W / m) * (wl.H / m) == pytest.approx(inside.sum(), rel=1e-12)
    rng = np.random.default_rng(0)
    ls, js = rng.integers(0, m, 48), rng.integers(0, m, 48)
    ls[:2], js[:2] = (0, m - 1), (0, m - 1)
    Ps = oracle.bin_density_at(wl.W, wl.H, *wl.arrays(), m, ls, js)
    assert np.abs(Ph[ls, js] - Ps).max() <= TOL * np.abs(Ph).max()
    us, ps = rng.integers(0, m, 24), rng.integers(0, m, 24)
    us[:3], ps[:3] = (0, 5, m - 1), (7, 0, m - 1)
    As = oracle.bin_coeffs_at(wl.W, wl.H, Ph, us, ps)
    assert np.abs(ah[us, ps] - As).max() <= TOL * np.abs(ah).max()
    # field at sampled bin centres from the same coefficients, by the point evaluation
    sl, sj = rng.integers(0, m, 12), rng.integers(0, m, 12)
    xc, yc = (sl + 0.5) * wl.W / m, (sj + 0.5) * wl.H / m
    ps_, ex, ey = oracle.point_field(wl.W, wl.H, ah, xc, yc)
    for got, want in ((psi, ps_), (xix, ex), (xiy, ey)):
        g = got.cpu().numpy()[sl, sj]
        assert np.abs(g - want).max() <= 1e-11 * np.abs(got.cpu().numpy()).max()
    # block values from the bins: sampled blocks (all macros among them) against the oracle
    N, gx, gy = pp.bin_interp(x, y, w, h, psi, xix, xiy, W=wl.W, H=wl.H)
    idx = np.concatenate([rng.choice(wl.n, 200, replace=False), np.argsort(wl.w * wl.h)[-20:]])
    arrs = [v[idx] for v in wl.arrays()]
    No, gxo, gyo = oracle.bin_interp(wl.W, wl.H, *arrs, m, psi.cpu().numpy(), xix.cpu().numpy(), xiy.cpu().numpy())
    for got, want in ((N, No), (gx, gxo), (gy, gyo)):
        g = got.cpu().numpy()
        assert np.abs(g[idx] - want).max() <= TOL * np.abs(g).max()
