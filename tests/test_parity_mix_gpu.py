"""GPU parity of the mixed split (PP_BF16MIX) against the FP64 oracle.

The mixed split contracts the low-frequency tiles with the bf16 hi/lo split (three products) and the
others with hi only (one product): per axis the first ceil(M / 1024) tiles of 256 frequencies, the
coefficient contraction on the tiles with u and p both in that corner, the gradient contraction of gx
(gy) on the N tiles of u (p) in it.  Its checks:

* the workload's own coefficients (the case the split is made for, Sec. III-A: they fall like
  1 / (u^2 + p^2)): E, a and g against the oracle at the split-precision bar (1e-3), and no more than
  MIX_FACTOR times the full split's own error on the same input (both run here);
* each part at its own precision: the raw block sums a / f in the three-product corner per 64 x 64
  tile at the bf16x3 bar and elsewhere at the bf16 bar; gradients of flat-spectrum coefficients
  restricted to the three-product N tiles at the bf16x3 bar, restricted to the others at the bf16 bar
  (so a wrong N-tile range or a corner tile contracted by the wrong kernel shows);
* the 2,000,500-block workload: three sampled coefficients in every 256 x 256 tile, scaled by
  f_up sum_i |S'_iu T'_ip| (bf16x3 sample bar in the corner, the per-term bf16 bound elsewhere), and the
  restricted flat-spectrum gradients at sampled blocks.
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
TOL_X3, TOL_BF16 = 1e-3, 3e-2          # the bars of tests/test_parity_bf16_gpu.py
MIX_FACTOR = 10.0
SAMPLE_TOL_X3 = 1e-5                   # as tests/test_workloads_gpu.py for bf16x3
SAMPLE_TOL_BF16 = 4e-3                 # per-term bound of one bf16 product: (2 * 2^-9 + 2^-18) |xy|


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def mix_tiles(M):
    """The three-product tiles per axis, as include/pplace.h documents them."""
    return min(max(1, -(-M // 1024)), -(-M // 256))


def corner(Mu, Mp):
    return 256 * mix_tiles(Mu), 256 * mix_tiles(Mp)


def region_tile_max(A, B, cu, cp, inside):
    """Worst 64 x 64 tile relative error over the tiles inside (or outside) the corner [0, cu) x [0, cp)."""
    worst = 0.0
    big = max(float(np.linalg.norm(B[u0:u0 + 64, p0:p0 + 64]))
              for u0 in range(0, B.shape[0], 64) for p0 in range(0, B.shape[1], 64))
    for u0 in range(0, B.shape[0], 64):
        for p0 in range(0, B.shape[1], 64):
            if (u0 < cu and p0 < cp) != inside:
                continue
            nb = float(np.linalg.norm(B[u0:u0 + 64, p0:p0 + 64]))
            d = float(np.linalg.norm(A[u0:u0 + 64, p0:p0 + 64] - B[u0:u0 + 64, p0:p0 + 64]))
            worst = max(worst, d / (nb if nb > 0 else (big if big > 0 else 1.0)))
    return worst


def restricted_flat(wl, seed):
    """Flat-spectrum coefficient sets for the gradients restricted to the three-product N tiles and
    to the others: gx's N axis is u, gy's is p."""
    a_x, a_y = parity.flat_field_coeffs(wl.W, wl.H, wl.Mu, wl.Mp, seed)
    cu, cp = corner(wl.Mu, wl.Mp)
    u = np.arange(wl.Mu)[:, None]
    p = np.arange(wl.Mp)[None, :]
    return {"x3": (np.where(u < cu, a_x, 0.0), np.where(p < cp, a_y, 0.0)),
            "bf16": (np.where(u >= cu, a_x, 0.0), np.where(p >= cp, a_y, 0.0))}


SHAPES = [
    (3001, 300, 150, 500.0, 300.0, 3),
    (5000, 257, 513, 300.0, 900.0, 4),
    (2000, 1100, 600, 2000.0, 1000.0, 6),
    (1500, 2100, 300, 3000.0, 400.0, 7),
]


@pytest.mark.parametrize("n,Mu,Mp,W,H,seed", SHAPES)
def test_mix_parity(n, Mu, Mp, W, H, seed):
    wl = make_random(n, W, H, Mu, Mp, seed=seed)
    cu, cp = corner(Mu, Mp)
    say(f"[mix] {wl.name} n={n} Mu={Mu} Mp={Mp}: three products on u < {cu}, p < {cp}")
    ref = gpu_parity.OracleRef(wl)
    E, a, gx, gy = gpu_parity.run_gpu(wl, "bf16mix")
    e = gpu_parity.errors(ref, E, a, gx, gy)
    E3, a3, gx3, gy3 = gpu_parity.run_gpu(wl, "bf16x3")
    e3 = gpu_parity.errors(ref, E3, a3, gx3, gy3)
    own = {k: e[k] for k in ("E", "a", "g", "g_tile")}
    say("   mix " + " ".join(f"{k}={v:.2e}" for k, v in own.items()) + " | bf16x3 "
        + " ".join(f"{k}={e3[k]:.2e}" for k in own))
    for k, v in own.items():
        assert v <= TOL_X3, (k, v)
        assert v <= MIX_FACTOR * max(e3[k], 1e-7), (k, v, e3[k])
    # coefficients part by part: raw block sums per 64 x 64 tile
    R = parity.raw_from_coeffs(a, ref.f)
    Rr = np.where(ref.f != 0, ref.R, 0.0)
    t_in, t_out = region_tile_max(R, Rr, cu, cp, True), region_tile_max(R, Rr, cu, cp, False)
    say(f"   raw block sums: corner tiles {t_in:.2e}, other tiles {t_out:.2e}")
    assert t_in <= TOL_X3 and t_out <= TOL_BF16
    # gradients part by part
    x, y, w, h = gpu_parity.dev(*wl.arrays())
    for part, (cx, cy) in restricted_flat(wl, 23).items():
        gxo, _ = oracle.grad(wl.W, wl.H, *wl.arrays(), cx)
        _, gyo = oracle.grad(wl.W, wl.H, *wl.arrays(), cy)
        gxg, _ = pp.field(x, y, w, h, gpu_parity.dev(cx)[0], W=wl.W, H=wl.H, precision="bf16mix")
        _, gyg = pp.field(x, y, w, h, gpu_parity.dev(cy)[0], W=wl.W, H=wl.H, precision="bf16mix")
        torch.cuda.synchronize()
        errs = {"gx": parity.rel(gxg.cpu().numpy(), gxo), "gy": parity.rel(gyg.cpu().numpy(), gyo),
                "gx_tile": parity.row_tile_rel_max(gxg.cpu().numpy(), gxo),
                "gy_tile": parity.row_tile_rel_max(gyg.cpu().numpy(), gyo)}
        say(f"   flat-spectrum gradients on the {part} N tiles: " + " ".join(f"{k}={v:.2e}" for k, v in errs.items()))
        assert max(errs.values()) <= (TOL_X3 if part == "x3" else TOL_BF16), (part, errs)


def test_mix_small_problems_equal_the_full_split():
    """At most one tile of 256 frequencies per axis the corner is the whole plane: PP_BF16MIX runs the
    three-product kernels alone and gives the PP_BF16X3 results bit for bit."""
    wl = make_random(2000, 200.0, 150.0, 200, 96, seed=9)
    m = gpu_parity.run_gpu(wl, "bf16mix")
    f = gpu_parity.run_gpu(wl, "bf16x3")
    assert m[0] == f[0]
    for u, v in zip(m[1:], f[1:]):
        assert np.array_equal(u, v)


def test_mix_edges_determinism_and_autograd():
    say("[mix] n=0, determinism, autograd, rejected rows")
    x0 = torch.empty(0, dtype=torch.float64, device=DEV)
    E, a = pp.energy(x0, x0, x0, x0, W=10.0, H=10.0, Mu=1300, Mp=9, precision="bf16mix")
    assert float(E.cpu()) == 0.0 and float(a.abs().max().cpu()) == 0.0
    wl = make_random(20000, 700.0, 500.0, 1300, 600, seed=21, wmax=8, hmax=2)
    runs = [gpu_parity.run_gpu(wl, "bf16mix") for _ in range(2)]
    assert runs[0][0] == runs[1][0]
    for u, v in zip(runs[0][1:], runs[1][1:]):
        assert np.array_equal(u, v)
    wl = make_random(500, 600.0, 400.0, 700, 300, seed=31)
    xs, ys, ws, hs = gpu_parity.dev(*wl.arrays())
    xr, yr = xs.clone().requires_grad_(True), ys.clone().requires_grad_(True)
    E = pp.energy_autograd(xr, yr, ws, hs, W=wl.W, H=wl.H, Mu=wl.Mu, Mp=wl.Mp, precision="bf16mix")
    E.backward()
    _, a = pp.energy(xs, ys, ws, hs, W=wl.W, H=wl.H, Mu=wl.Mu, Mp=wl.Mp, precision="bf16mix")
    gx, gy = pp.field(xs, ys, ws, hs, a, W=wl.W, H=wl.H, precision="bf16mix")
    assert torch.equal(xr.grad, gx) and torch.equal(yr.grad, gy)
    with pytest.raises(pp.PPError):
        pp.point_field(xs, ys, a, W=wl.W, H=wl.H, precision="bf16mix")


def test_mix_bench_workload_cells2m_macros500_M2048():
    wl = make_config(4)
    cu, cp = corner(wl.Mu, wl.Mp)
    say(f"[mix workload] {wl.name} n={wl.n} M={wl.Mu}x{wl.Mp}: three products on u < {cu}, p < {cp}")
    x, y, w, h = (torch.as_tensor(v, device=DEV) for v in wl.arrays())
    ws = torch.empty(pp.workspace_size(wl.W, wl.H, wl.n, wl.Mu, wl.Mp, precision="bf16mix"), dtype=torch.uint8,
                     device=DEV)
    E, a = pp.energy(x, y, w, h, W=wl.W, H=wl.H, Mu=wl.Mu, Mp=wl.Mp, precision="bf16mix", workspace=ws)
    torch.cuda.synchronize()
    an = a.cpu().numpy()
    us, ps = parity.samples_per_tile(wl.Mu, wl.Mp, 3, 4)
    ao, _, Rabs = oracle.coeffs_sampled_full(wl.W, wl.H, *wl.arrays(), us, ps)
    f = oracle.coef_factors(wl.W, wl.H, wl.Mu, wl.Mp)[us, ps]
    errs = parity.scaled_sample_errors(an[us, ps], ao, f, Rabs)
    inside = (us < cu) & (ps < cp)
    worst_in, worst_out = float(errs[inside].max()), float(errs[~inside].max())
    say(f"   {len(us)} sampled coefficients: corner worst scaled error {worst_in:.2e}, elsewhere {worst_out:.2e}")
    assert worst_in <= SAMPLE_TOL_X3 and worst_out <= SAMPLE_TOL_BF16
    idx = np.unique(np.concatenate([np.random.default_rng(44).choice(wl.n, 48, replace=False),
                                    np.argsort(wl.w * wl.h)[-16:]]))
    for part, (cx, cy) in restricted_flat(wl, 44).items():
        gxo, _ = oracle.grad_sampled(wl.W, wl.H, *wl.arrays(), cx, idx)
        _, gyo = oracle.grad_sampled(wl.W, wl.H, *wl.arrays(), cy, idx)
        gx, _ = pp.field(x, y, w, h, torch.as_tensor(cx, device=DEV), W=wl.W, H=wl.H, precision="bf16mix",
                         workspace=ws)
        _, gy = pp.field(x, y, w, h, torch.as_tensor(cy, device=DEV), W=wl.W, H=wl.H, precision="bf16mix",
                         workspace=ws)
        torch.cuda.synchronize()
        eg = (parity.rel(gx.cpu().numpy()[idx], gxo), parity.rel(gy.cpu().numpy()[idx], gyo))
        say(f"   flat-spectrum gradients on the {part} N tiles at {len(idx)} blocks: gx {eg[0]:.2e} gy {eg[1]:.2e}")
        assert max(eg) <= (TOL_X3 if part == "x3" else TOL_BF16), (part, eg)
