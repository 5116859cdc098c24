"""GPU parity of the evaluation entry points against the FP64 oracle.

* pp_point_field: psi and the field xi = -grad psi at arbitrary points (eq. psi, eq. ksi), at the
  block centres and on a grid, FP64 (1e-10 relative), FP32 (1e-5 relative; the FP32 operand
  rounding argument of the FP32 parity tests applies unchanged), BF16X3 (1e-3, the split-precision
  bar) and plain BF16 (3e-2).
* pp_block_potential: N_i, the integral of psi over block i (Sec. II-B with the exact density),
  against the oracle and through the identity E = 1/2 sum_i N_i against pp_energy.
"""
import sys

import numpy as np
import pytest

import oracle
from tests import parity
from workloads import make_config, make_random

torch = pytest.importorskip("torch")
pp = pytest.importorskip("paper_2307_12041_amd")

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
TOL = {"fp64": 1e-10, "fp32": 1e-5, "bf16x3": 1e-3, "bf16": 3e-2}


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def dev(*arrs):
    return [torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device=DEV) for a in arrs]


def rel(a, b):
    nb = np.linalg.norm(np.ravel(b))
    return np.linalg.norm(np.ravel(a) - np.ravel(b)) / (nb if nb > 0 else 1.0)


def coeffs_of(wl):
    """FP64 oracle coefficients (inputs of the evaluation calls come from the oracle, not the GPU)."""
    _, a, _ = oracle.energy(wl.W, wl.H, *wl.arrays(), wl.Mu, wl.Mp)
    return a


SHAPES = [
    (1, 5, 3, 10.0, 7.0, 0),
    (37, 24, 20, 100.0, 60.0, 1),
    (1000, 64, 64, 1024.0, 1024.0, 2),
    (3001, 300, 150, 500.0, 300.0, 3),
    (4100, 129, 257, 300.0, 900.0, 4),
]


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3", "bf16"])
@pytest.mark.parametrize("n,Mu,Mp,W,H,seed", SHAPES)
def test_point_field_at_centres(prec, n, Mu, Mp, W, H, seed):
    """The real (decaying) coefficients of the blocks, and flat-spectrum ones (every frequency tile
    weighs alike), each over all points and per tile of 256 points."""
    wl = make_random(n, W, H, Mu, Mp, seed=seed)
    say(f"[point field] {wl.name} n={n} Mu={Mu} Mp={Mp} prec={prec}")
    x, y, _, _ = dev(*wl.arrays())
    for kind, a in (("real", coeffs_of(wl)), ("flat", parity.flat_point_coeffs(Mu, Mp, seed + 100))):
        psi, ex, ey = pp.point_field(x, y, dev(a)[0], W=W, H=H, precision=prec)
        torch.cuda.synchronize()
        po, exo, eyo = oracle.point_field(W, H, a, wl.x, wl.y)
        got = (psi.cpu().numpy(), ex.cpu().numpy(), ey.cpu().numpy())
        errs = [rel(g, r) for g, r in zip(got, (po, exo, eyo))]
        errs += [parity.row_tile_rel_max(g, r) for g, r in zip(got, (po, exo, eyo))]
        say(f"   {kind}: rel err psi={errs[0]:.3e} xix={errs[1]:.3e} xiy={errs[2]:.3e}; worst 256-point tile "
            f"{max(errs[3:]):.3e}")
        assert max(errs) <= TOL[prec], (kind, errs)


@pytest.mark.parametrize("prec", ["fp64", "bf16x3"])
def test_point_field_on_grid_and_partial_outputs(prec):
    """psi on a ragged grid of points (a picture of the potential), and each output alone equals the
    same output computed with the others."""
    wl = make_random(600, 200.0, 120.0, 96, 70, seed=13, wmax=20.0, hmax=10.0)
    a = coeffs_of(wl)
    gx, gy = np.meshgrid(np.linspace(0.0, wl.W, 131), np.linspace(0.0, wl.H, 77), indexing="ij")
    px, py = gx.ravel(), gy.ravel()
    say(f"[point field] grid {px.size} points, Mu={wl.Mu} Mp={wl.Mp} prec={prec}")
    tpx, tpy, ta = dev(px, py, a)
    psi, ex, ey = pp.point_field(tpx, tpy, ta, W=wl.W, H=wl.H, precision=prec)
    po, exo, eyo = oracle.point_field(wl.W, wl.H, a, px, py)
    errs = (rel(psi.cpu().numpy(), po), rel(ex.cpu().numpy(), exo), rel(ey.cpu().numpy(), eyo))
    say(f"   rel err psi={errs[0]:.3e} xix={errs[1]:.3e} xiy={errs[2]:.3e}")
    assert max(errs) <= TOL[prec], errs
    for want in (("psi",), ("xix",), ("xiy",), ("psi", "xiy"), ("xix", "xiy")):
        outs = pp.point_field(tpx, tpy, ta, W=wl.W, H=wl.H, want=want, precision=prec)
        for name, full, got in zip(("psi", "xix", "xiy"), (psi, ex, ey), outs):
            if name in want:
                assert torch.equal(got, full), (want, name)
            else:
                assert got is None


def test_point_field_zero_points():
    e = torch.empty(0, dtype=torch.float64, device=DEV)
    a = torch.zeros((8, 6), dtype=torch.float64, device=DEV)
    psi, ex, ey = pp.point_field(e, e, a, W=5.0, H=3.0)
    assert psi.numel() == 0 and ex.numel() == 0 and ey.numel() == 0


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3", "bf16"])
@pytest.mark.parametrize("n,Mu,Mp,W,H,seed", SHAPES)
def test_block_potential(prec, n, Mu, Mp, W, H, seed):
    """Real coefficients and flat-spectrum ones (the operand a_up / (wt_u vt_p) ~N(0, 1)), each over
    all blocks and per tile of 256 blocks."""
    wl = make_random(n, W, H, Mu, Mp, seed=seed)
    say(f"[block potential] {wl.name} n={n} Mu={Mu} Mp={Mp} prec={prec}")
    x, y, w, h = dev(*wl.arrays())
    for kind, a in (("real", coeffs_of(wl)), ("flat", parity.flat_potential_coeffs(W, H, Mu, Mp, seed + 200))):
        N = pp.block_potential(x, y, w, h, dev(a)[0], W=W, H=H, precision=prec).cpu().numpy()
        No = oracle.block_potential(W, H, *wl.arrays(), a)
        e, et = rel(N, No), parity.row_tile_rel_max(N, No)
        say(f"   {kind}: rel err N={e:.3e}, worst 256-block tile {et:.3e}")
        assert e <= TOL[prec] and et <= TOL[prec], (kind, e, et)


def test_block_potential_overhanging_and_energy_identity():
    wl = make_random(800, 400.0, 300.0, 96, 80, seed=8, wmax=60.0, hmax=40.0, inside=False)
    say(f"[block potential] {wl.name} overhanging; 1/2 sum N = E")
    x, y, w, h = dev(*wl.arrays())
    E, a = pp.energy(x, y, w, h, W=wl.W, H=wl.H, Mu=wl.Mu, Mp=wl.Mp, precision="fp64")
    N = pp.block_potential(x, y, w, h, a, W=wl.W, H=wl.H)
    No = oracle.block_potential(wl.W, wl.H, *wl.arrays(), a.cpu().numpy())
    assert rel(N.cpu().numpy(), No) <= TOL["fp64"]
    Ev = float(E.cpu())
    assert abs(0.5 * float(N.sum().cpu()) - Ev) <= 1e-10 * abs(Ev)


def test_evaluation_at_full_size_cells2m_macros500_M2048():
    """At 2,000,500 blocks and 2048 x 2048 frequencies, FP64 and BF16X3 evaluation of the FP64
    coefficients and of flat-spectrum coefficients (every 256 x 256 frequency tile weighs alike):
    psi and xi at 256 sampled block centres against the oracle, the block potentials of 64 sampled
    blocks against the oracle, and (real coefficients) 1/2 sum_i N_i against the energy over all
    blocks."""
    wl = make_config(4)
    say(f"[evaluation] {wl.name} n={wl.n} Mu={wl.Mu} Mp={wl.Mp}")
    x, y, w, h = dev(*wl.arrays())
    E, a = pp.energy(x, y, w, h, W=wl.W, H=wl.H, Mu=wl.Mu, Mp=wl.Mp, precision="fp64")
    torch.cuda.synchronize()
    an = a.cpu().numpy()
    Ev = float(E.cpu())
    rng = np.random.default_rng(4)
    idx = np.sort(rng.choice(wl.n, 256, replace=False))
    jdx = np.sort(rng.choice(wl.n, 64, replace=False))
    sets = {"real": (an, an), "flat": (parity.flat_point_coeffs(wl.Mu, wl.Mp, 41),
                                       parity.flat_potential_coeffs(wl.W, wl.H, wl.Mu, wl.Mp, 43))}
    for kind, (apt, apot) in sets.items():
        po, exo, eyo = oracle.point_field(wl.W, wl.H, apt, wl.x[idx], wl.y[idx])
        No = oracle.block_potential(wl.W, wl.H, wl.x[jdx], wl.y[jdx], wl.w[jdx], wl.h[jdx], apot)
        tpt, tpot = (a, a) if kind == "real" else dev(apt, apot)
        for prec, tol_id in (("fp64", 1e-10), ("bf16x3", 1e-3)):
            psi, ex, ey = pp.point_field(x, y, tpt, W=wl.W, H=wl.H, precision=prec)
            N = pp.block_potential(x, y, w, h, tpot, W=wl.W, H=wl.H, precision=prec)
            torch.cuda.synchronize()
            errs = (rel(psi.cpu().numpy()[idx], po), rel(ex.cpu().numpy()[idx], exo),
                    rel(ey.cpu().numpy()[idx], eyo))
            eN = rel(N.cpu().numpy()[jdx], No)
            say(f"   {kind} {prec}: sampled point field rel err psi={errs[0]:.3e} xix={errs[1]:.3e} "
                f"xiy={errs[2]:.3e}; sampled N {eN:.3e}")
            assert max(errs) <= TOL[prec] and eN <= TOL[prec], (kind, prec, errs, eN)
            if kind == "real":
                eE = abs(0.5 * float(N.sum().cpu()) - Ev) / abs(Ev)
                say(f"   |1/2 sum N - E| / E = {eE:.3e}")
                assert eE <= tol_id, (prec, eE)
