"""The tile-resolving parity metrics see every output tile (CPU only, on oracle outputs).

A GPU result that is right in the first tile and wrong or missing in any other one must fail the
parity tests.  Here the "wrong result" is planted in oracle outputs: one tile of coefficients is
zeroed, one tile of the gradient operand is dropped, one tile of blocks is zeroed, and at full
size each sampled coefficient is replaced by zero.  Every new metric must then exceed the bf16x3
bar of 1e-3 (the scaled full-size samples their bar of 1e-5), whereas the old whole-array norms,
kept here to show why they were replaced, stay below it for the coefficients and the gradient of
real (decaying) coefficients.
"""
import numpy as np
import pytest

import oracle
from tests import parity
from workloads import make_config, make_random

BAR = 1e-3          # bf16x3 bar of the parity tests
SAMPLE_BAR = 1e-5   # bf16x3 bar of the scaled full-size sample errors

SHAPES = [(5000, 257, 513, 300.0, 900.0, 4), (3001, 300, 150, 500.0, 300.0, 3)]


@pytest.mark.parametrize("n,Mu,Mp,W,H,seed", SHAPES)
def test_zeroing_any_coefficient_tile_fails_the_tile_metric(n, Mu, Mp, W, H, seed):
    wl = make_random(n, W, H, Mu, Mp, seed=seed)
    a, _ = oracle.coeffs(W, H, *wl.arrays(), Mu, Mp)
    R = oracle.raw_moments(W, H, *wl.arrays(), Mu, Mp)
    f = oracle.coef_factors(W, H, Mu, Mp)
    base = parity.coeff_errors(a, R, f)
    assert base["flat_tile"] < 1e-12          # the oracle's own a reproduces its raw sums
    blind = []
    for u0 in range(0, Mu, 256):
        for p0 in range(0, Mp, 256):
            if u0 == 0 and p0 == 0:
                continue
            bad = a.copy()
            bad[u0:u0 + 256, p0:p0 + 256] = 0.0
            e = parity.coeff_errors(bad, R, f)
            assert e["flat_tile"] > BAR, (u0, p0, e)
            blind.append(parity.rel(bad, a))
    # the whole-array norm of a cannot see these tiles
    assert max(blind) < BAR, blind


@pytest.mark.parametrize("n,Mu,Mp,W,H,seed", SHAPES)
def test_dropping_any_gradient_tile_fails_with_flat_coefficients(n, Mu, Mp, W, H, seed):
    wl = make_random(n, W, H, Mu, Mp, seed=seed)
    a_x, a_y = parity.flat_field_coeffs(W, H, Mu, Mp, seed)
    gx, _ = oracle.grad(W, H, *wl.arrays(), a_x)
    _, gy = oracle.grad(W, H, *wl.arrays(), a_y)
    a_real, _ = oracle.coeffs(W, H, *wl.arrays(), Mu, Mp)
    gxr, gyr = oracle.grad(W, H, *wl.arrays(), a_real)
    blind = []
    # a dropped 256-wide tile of the summed (K) or of the output (N) frequencies of each contraction
    for axis, M in ((0, Mu), (1, Mp)):
        for k0 in range(0, M, 256):
            sl = (slice(k0, k0 + 256), slice(None)) if axis == 0 else (slice(None), slice(k0, k0 + 256))
            bx, by = a_x.copy(), a_y.copy()
            bx[sl] = 0.0
            by[sl] = 0.0
            gxb, _ = oracle.grad(W, H, *wl.arrays(), bx)
            _, gyb = oracle.grad(W, H, *wl.arrays(), by)
            ex, ey = parity.rel(gxb, gx), parity.rel(gyb, gy)
            assert ex > BAR and ey > BAR, (axis, k0, ex, ey)
            if k0 > 0:
                br = a_real.copy()
                br[sl] = 0.0
                gxrb, gyrb = oracle.grad(W, H, *wl.arrays(), br)
                blind.append(parity.rel(np.concatenate([gxrb, gyrb]), np.concatenate([gxr, gyr])))
    assert max(blind) < BAR, blind
    # a dropped tile of blocks
    g = np.stack([gx, gy], axis=1)
    for i0 in range(0, n, parity.ROW_TILE):
        bad = g.copy()
        bad[i0:i0 + parity.ROW_TILE] = 0.0
        assert parity.row_tile_rel_max(bad, g) >= 1.0


def test_flat_point_and_potential_coefficients_weigh_every_tile():
    """The evaluation rows with flat coefficients: dropping any 64-wide frequency tile of a moves
    psi, xi and the block potentials by more than the bar."""
    n, Mu, Mp, W, H = 600, 200, 150, 300.0, 200.0
    wl = make_random(n, W, H, Mu, Mp, seed=9)
    ap = parity.flat_point_coeffs(Mu, Mp, 1)
    an = parity.flat_potential_coeffs(W, H, Mu, Mp, 2)
    ref = oracle.point_field(W, H, ap, wl.x, wl.y)
    Nref = oracle.block_potential(W, H, *wl.arrays(), an)
    for axis, M in ((0, Mu), (1, Mp)):
        for k0 in range(0, M, 64):
            sl = (slice(k0, k0 + 64), slice(None)) if axis == 0 else (slice(None), slice(k0, k0 + 64))
            bp, bn = ap.copy(), an.copy()
            bp[sl] = 0.0
            bn[sl] = 0.0
            got = oracle.point_field(W, H, bp, wl.x, wl.y)
            for r, gv in zip(ref, got):
                assert parity.rel(gv, r) > BAR, (axis, k0)
            assert parity.rel(oracle.block_potential(W, H, *wl.arrays(), bn), Nref) > BAR, (axis, k0)


def test_samples_cover_every_kernel_tile():
    us, ps = parity.samples_per_tile(4096, 2048, 3, 0)
    tiles = {(u // 256, p // 256) for u, p in zip(us, ps)}
    assert len(tiles) == 16 * 8 and len(us) == 3 * 16 * 8
    assert not np.any((us == 0) & (ps == 0))
    us, ps = parity.samples_per_tile(300, 150, 4, 1)
    assert {(u // 256, p // 256) for u, p in zip(us, ps)} == {(0, 0), (1, 0)}


def test_full_size_samples_see_a_zeroed_tile():
    """At the 2,000,500-block workload (M = 2048 x 2048), a coefficient replaced by zero is
    |R| / sum|S'T'| ~ n^-1/2 away from the oracle in the scaled metric: far above the 1e-5 bar in
    the worst sample of every 256 x 256 tile."""
    wl = make_config(4)
    us, ps = parity.samples_per_tile(wl.Mu, wl.Mp, 4, 7)
    a, R, Rabs = oracle.coeffs_sampled_full(wl.W, wl.H, *wl.arrays(), us, ps)
    f = oracle.coef_factors(wl.W, wl.H, wl.Mu, wl.Mp)[us, ps]
    assert np.allclose(f * R, a, rtol=1e-13, atol=0)
    errs = parity.scaled_sample_errors(np.zeros_like(a), a, f, Rabs)
    per_tile = parity.tile_max_of_samples(errs, us, ps)
    assert len(per_tile) == 64
    assert min(per_tile.values()) > SAMPLE_BAR, min(per_tile.values())
