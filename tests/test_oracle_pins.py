"""Pins of the FP64 oracle against facts the paper and the mathematics fix (CPU only).

Each test checks the oracle against something other than itself: a closed form, a library
routine the method reduces to, an independent PDE solve, an exact invariant, or a finite
difference.  Together they are chosen so that a dropped term, a wrong constant, sign, index
or a transposed operand anywhere in the oracle fails at least one of them:

  coefficient constants / three cases ... strips (closed form), DCT-II special case, FD Poisson
  (0,0) handling and mean subtraction ... compatibility, tiling
  energy normalisation ................ strips, FD Poisson
  truncation semantics ................ monotone energy, O(M^-3) convergence
  gradient ............................ central differences, mirror signs, field quadrature
  point potential / field ............. block quadrature of psi, finite differences of psi
  bin scheme .......................... lattice brute force, DCT-II / DCT-III, whole-bin blocks,
                                        adjoint of the densities, convergence to the direct path
"""
import numpy as np
import pytest
import scipy.fft
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import oracle
from workloads import make_random

PI = np.pi


def _E(W, H, x, y, w, h, Mu, Mp):
    return oracle.energy(W, H, x, y, w, h, Mu, Mp)[0]


# ---------------------------------------------------------------------------------------------
# Closed form: a block spanning the full height is a 1-D problem.  With rho(x) = theta(x) - c,
# c = w/W, the Neumann solution has psi' = F, F(x) = -int_0^x rho, and E = (H/2) int_0^W F^2.
# For alpha = x0 - w/2, beta = x0 + w/2:
#   E_inf = (H/2) [c^2 alpha^3/3 + (c^3 alpha^3 + (w - c beta)^3)/(3(1-c)) + c^2 (W-beta)^3/3].
# Only the u-row (p = 0) of the series is non-zero, so this pins a_{u,0} (eq. au0) and the
# energy normalisation; the transposed strip pins a_{0,p} (eq. a0p).
# ---------------------------------------------------------------------------------------------
def strip_energy(L, Hperp, w, x0):
    c = w / L
    al, be = x0 - w / 2, x0 + w / 2
    return (Hperp / 2) * (c * c * al**3 / 3 + (c**3 * al**3 + (w - c * be) ** 3) / (3 * (1 - c))
                          + c * c * (L - be) ** 3 / 3)


def test_strip_closed_form_and_cubic_convergence():
    W, H, w, x0 = 10.0, 3.0, 2.5, 3.7
    Einf = strip_energy(W, H, w, x0)
    assert Einf == pytest.approx(5.97890625, rel=1e-12)
    errs = []
    for M in (16, 64, 256, 1024):
        E = _E(W, H, [x0], [H / 2], [w], [H], M, 5)
        assert E <= Einf * (1 + 1e-14)
        errs.append((Einf - E) / Einf)
    assert errs[-1] < 3e-9
    # tail of sum_u a_u0 I_u0 ~ sum u^-4 -> O(M^-3): a 4x larger M cuts the error ~64x
    for e0, e1 in zip(errs, errs[1:]):
        assert 40 < e0 / e1 < 90


def test_strip_transposed_pins_a0p():
    W, H, h, y0 = 4.0, 9.0, 1.75, 6.2
    Einf = strip_energy(H, W, h, y0)
    E = _E(W, H, [W / 2], [y0], [W], [h], 3, 2048)
    assert E == pytest.approx(Einf, rel=2e-9)


def test_two_strips_interaction():
    # Two full-height strips: F is the sum of the two single-strip F's, so E is quadratic in
    # them; compare with direct quadrature of F^2 on a fine grid.
    W, H = 7.0, 2.0
    strips = [(1.0, 2.2), (0.6, 5.1)]
    xs = np.linspace(0, W, 700001)
    F = np.zeros_like(xs)
    for w, x0 in strips:
        c = w / W
        rho_int = np.clip(xs - (x0 - w / 2), 0, w) - c * xs   # int_0^x rho
        F -= rho_int
    Eq = 0.5 * H * np.trapezoid(F * F, xs)
    E = _E(W, H, [s[1] for s in strips], [H / 2, H / 2], [s[0] for s in strips], [H, H], 4096, 3)
    assert E == pytest.approx(Eq, rel=1e-8)


# ---------------------------------------------------------------------------------------------
# Special case that reduces to a library routine: blocks that are exactly bins of an m x m
# grid.  Then the closed forms become the binned coefficients of Sec. III-D (eqs. disa-b..d),
# whose double sums are a 2-D DCT-II of the bin occupancy.  scipy's dctn(type=2) computes
# y[k,q] = 4 sum_l sum_j P_lj cos(pi k (2l+1)/(2m)) cos(pi q (2j+1)/(2m)).
# The garbled cosine argument of eq. disa-c is read as u (l + 1/2) pi / m (symmetry with b, d).
# ---------------------------------------------------------------------------------------------
@pytest.mark.parametrize("W,H,m", [(16.0, 16.0, 8), (12.0, 5.0, 6)])
def test_bin_blocks_match_dct2(W, H, m):
    rng = np.random.default_rng(7)
    P = rng.integers(0, 3, size=(m, m))           # 0, 1 or 2 stacked blocks per bin
    xs, ys = [], []
    for l in range(m):
        for j in range(m):
            for _ in range(P[l, j]):
                xs.append(W / m * (l + 0.5))
                ys.append(H / m * (j + 0.5))
    n = len(xs)
    wb, hb = W / m, H / m
    Mu = Mp = m
    a, _ = oracle.coeffs(W, H, np.array(xs), np.array(ys), np.full(n, wb), np.full(n, hb), Mu, Mp)
    D = scipy.fft.dctn(P.astype(float), type=2) / 4.0
    u = np.arange(Mu)[:, None].astype(float)
    p = np.arange(Mp)[None, :].astype(float)
    ref = np.zeros((Mu, Mp))
    uu, pp = np.meshgrid(np.arange(1, Mu), np.arange(1, Mp), indexing="ij")
    ref[1:, 1:] = (16 * W**2 * H**2 / (uu * pp * (uu**2 * H**2 + pp**2 * W**2) * PI**4)
                   * np.sin(uu * PI / (2 * m)) * np.sin(pp * PI / (2 * m)) * D[1:, 1:])
    pr = np.arange(1, Mp)
    ref[0, 1:] = 4 * H**2 / (pr**3 * PI**3 * m) * np.sin(pr * PI / (2 * m)) * D[0, 1:]
    ur = np.arange(1, Mu)
    ref[1:, 0] = 4 * W**2 / (ur**3 * PI**3 * m) * np.sin(ur * PI / (2 * m)) * D[1:, 0]
    del u, p
    scale = np.abs(ref).max()
    assert np.abs(a - ref).max() <= 1e-13 * scale
    assert a[0, 0] == 0.0


# ---------------------------------------------------------------------------------------------
# Independent PDE solve: cell-centred 5-point finite-volume Laplacian with zero-flux (Neumann)
# boundaries, exact cell-area density minus its mean, on a non-square region with block edges
# on cell faces.  E_h = 1/2 sum rho psi dA converges O(h^2); Richardson extrapolation of two
# grids must agree with the series energy (eq. psi coefficients, energy 1/2 iint rho psi).
# ---------------------------------------------------------------------------------------------
def _fd_poisson_energy(W, H, blocks, gx, gy):
    hx, hy = W / gx, H / gy
    xe = np.linspace(0, W, gx + 1)
    ye = np.linspace(0, H, gy + 1)
    rho = np.zeros((gx, gy))
    for (x0, y0, w, h) in blocks:
        ox = np.clip(np.minimum(xe[1:], x0 + w / 2) - np.maximum(xe[:-1], x0 - w / 2), 0, None)
        oy = np.clip(np.minimum(ye[1:], y0 + h / 2) - np.maximum(ye[:-1], y0 - h / 2), 0, None)
        rho += np.outer(ox, oy) / (hx * hy)
    rho -= rho.mean()

    def lap1d(g, hh):
        main = np.full(g, -2.0)
        main[0] = main[-1] = -1.0     # zero flux through the boundary face
        off = np.ones(g - 1)
        return sp.diags([off, main, off], [-1, 0, 1]) / hh**2

    A = sp.kron(lap1d(gx, hx), sp.identity(gy)) + sp.kron(sp.identity(gx), lap1d(gy, hy))
    A = A.tolil()
    b = -rho.ravel().copy()
    A[0, :] = 0
    A[0, 0] = 1.0                     # pin one value (the operator has constants in its kernel)
    b[0] = 0.0
    psi = spla.spsolve(A.tocsc(), b)
    return 0.5 * np.sum(rho.ravel() * psi) * hx * hy


def test_fd_poisson_energy_normalisation():
    W, H = 8.0, 6.0
    blocks = [(2.0, 2.0, 2.0, 1.0), (5.5, 4.0, 1.0, 3.0), (4.0, 4.5, 1.5, 0.5), (6.75, 1.25, 0.5, 0.5)]
    Es = oracle.energy(W, H, *map(np.array, zip(*blocks)), 1024, 768)[0]
    E1 = _fd_poisson_energy(W, H, blocks, 64, 48)
    E2 = _fd_poisson_energy(W, H, blocks, 128, 96)
    ER = (4 * E2 - E1) / 3
    assert abs(E2 - Es) / Es < 2e-2           # plain FD already close
    assert abs(ER - Es) / Es < 2e-4           # extrapolated: agrees to the O(h^4) remainder
    assert abs(ER - Es) < abs(E2 - Es)


# ---------------------------------------------------------------------------------------------
# Theorem 1 bounds on every coefficient.
# ---------------------------------------------------------------------------------------------
def test_theorem1_coefficient_bounds():
    wl = make_random(300, 50.0, 30.0, 40, 33, seed=3)
    a, _ = oracle.coeffs(wl.W, wl.H, *wl.arrays(), wl.Mu, wl.Mp)
    W, H, n = wl.W, wl.H, wl.n
    u = np.arange(1, wl.Mu)[:, None].astype(float)
    p = np.arange(1, wl.Mp)[None, :].astype(float)
    bup = 16 * W**2 * H**2 * n / (u * p * (u**2 * H**2 + p**2 * W**2) * PI**4)
    assert np.all(np.abs(a[1:, 1:]) <= bup)
    b0p = 4 * H**2 * wl.w.sum() / (p[0] ** 3 * PI**3 * W)
    bu0 = 4 * W**2 * wl.h.sum() / (u[:, 0] ** 3 * PI**3 * H)
    assert np.all(np.abs(a[0, 1:]) <= b0p)
    assert np.all(np.abs(a[1:, 0]) <= bu0)
    assert a[0, 0] == 0.0


# ---------------------------------------------------------------------------------------------
# Compatibility condition: a block covering the whole region only adds to the (0,0) moment,
# which the mean subtraction removes, so a, E and the other blocks' gradients do not change.
# ---------------------------------------------------------------------------------------------
def test_compatibility_full_cover_block():
    wl = make_random(40, 20.0, 12.0, 24, 20, seed=11)
    E0, a0, _ = oracle.energy(wl.W, wl.H, *wl.arrays(), wl.Mu, wl.Mp)
    g0 = oracle.grad(wl.W, wl.H, *wl.arrays(), a0)
    x, y, w, h = (np.append(v, e) for v, e in zip(wl.arrays(), (wl.W / 2, wl.H / 2, wl.W, wl.H)))
    E1, a1, _ = oracle.energy(wl.W, wl.H, x, y, w, h, wl.Mu, wl.Mp)
    g1 = oracle.grad(wl.W, wl.H, x, y, w, h, a1)
    assert E1 == pytest.approx(E0, rel=1e-13)
    assert np.abs(a1 - a0).max() <= 1e-13 * np.abs(a0).max()
    for k in range(2):
        assert np.abs(g1[k][:-1] - g0[k]).max() <= 1e-12 * np.abs(g0[k]).max()


def test_tiling_gives_zero_field():
    # 4 x 3 blocks tile [0,8] x [0,6] exactly: rho - mean = 0, so psi = 0, E = 0, g = 0.
    W, H = 8.0, 6.0
    xs, ys = np.meshgrid(np.arange(4) * 2 + 1.0, np.arange(3) * 2 + 1.0, indexing="ij")
    n = xs.size
    E, a, I = oracle.energy(W, H, xs.ravel(), ys.ravel(), np.full(n, 2.0), np.full(n, 2.0), 32, 32)
    gx, gy = oracle.grad(W, H, xs.ravel(), ys.ravel(), np.full(n, 2.0), np.full(n, 2.0), a)
    assert abs(E) < 1e-26
    assert np.abs(a).max() < 1e-13
    assert max(np.abs(gx).max(), np.abs(gy).max()) < 1e-12


# ---------------------------------------------------------------------------------------------
# Single rectangle: the moments are an outer product (rank one); a block centred in the region
# has zero odd-index coefficients and zero force.
# ---------------------------------------------------------------------------------------------
def test_single_rectangle_rank_one_and_centred_symmetry():
    W, H = 9.0, 7.0
    a, I = oracle.coeffs(W, H, [3.1], [4.4], [1.3], [0.7], 16, 12)
    J = I.copy()
    J[0, 0] = 0.7 * 1.3  # the raw (0,0) moment is w*h before the mean subtraction
    s = np.linalg.svd(J, compute_uv=False)
    assert s[1] <= 1e-13 * s[0]
    E, a, I = oracle.energy(W, H, [W / 2], [H / 2], [1.3], [0.7], 16, 12)
    assert np.abs(a[1::2, :]).max() < 1e-14 * np.abs(a).max()
    assert np.abs(a[:, 1::2]).max() < 1e-14 * np.abs(a).max()
    gx, gy = oracle.grad(W, H, [W / 2], [H / 2], [1.3], [0.7], a)
    assert abs(gx[0]) < 1e-13 and abs(gy[0]) < 1e-13


# ---------------------------------------------------------------------------------------------
# Mirror and transpose symmetries of the cosine basis.
# ---------------------------------------------------------------------------------------------
def test_mirror_and_transpose():
    wl = make_random(25, 30.0, 18.0, 20, 14, seed=5)
    W, H = wl.W, wl.H
    x, y, w, h = wl.arrays()
    E, a, _ = oracle.energy(W, H, x, y, w, h, wl.Mu, wl.Mp)
    gx, gy = oracle.grad(W, H, x, y, w, h, a)
    gsc = max(np.abs(gx).max(), np.abs(gy).max())
    Em, am, _ = oracle.energy(W, H, W - x, y, w, h, wl.Mu, wl.Mp)
    gxm, gym = oracle.grad(W, H, W - x, y, w, h, am)
    assert Em == pytest.approx(E, rel=1e-13)
    assert np.abs(gxm + gx).max() < 1e-11 * gsc
    assert np.abs(gym - gy).max() < 1e-11 * gsc
    uu = np.arange(wl.Mu)[:, None]
    assert np.abs(am - a * (-1.0) ** uu).max() < 1e-12 * np.abs(a).max()
    Ey, ay, _ = oracle.energy(W, H, x, H - y, w, h, wl.Mu, wl.Mp)
    gxy, gyy = oracle.grad(W, H, x, H - y, w, h, ay)
    assert Ey == pytest.approx(E, rel=1e-13)
    assert np.abs(gxy - gx).max() < 1e-11 * gsc
    assert np.abs(gyy + gy).max() < 1e-11 * gsc
    # transpose: swap the axes (and W/H, Mu/Mp): coefficients transpose, forces swap
    Et, at, _ = oracle.energy(H, W, y, x, h, w, wl.Mp, wl.Mu)
    gxt, gyt = oracle.grad(H, W, y, x, h, w, at)
    assert Et == pytest.approx(E, rel=1e-13)
    assert np.abs(at - a.T).max() < 1e-12 * np.abs(a).max()
    assert np.abs(gxt - gy).max() < 1e-11 * gsc and np.abs(gyt - gx).max() < 1e-11 * gsc


# ---------------------------------------------------------------------------------------------
# Truncation: E = 1/2 sum s_up A_up^2 is a sum of non-negative terms, so E >= 0 and E grows
# with Mu and with Mp.
# ---------------------------------------------------------------------------------------------
def test_energy_nonnegative_and_monotone_in_truncation():
    wl = make_random(60, 40.0, 40.0, 0, 0, seed=9)
    prev = -1.0
    for M in (2, 4, 8, 16, 32, 64):
        E = _E(wl.W, wl.H, *wl.arrays(), M, M)
        assert E >= prev
        prev = E
    Es = [_E(wl.W, wl.H, *wl.arrays(), 8, mp) for mp in (1, 3, 9, 27)]
    assert all(e0 <= e1 for e0, e1 in zip(Es, Es[1:])) and Es[0] >= 0


# ---------------------------------------------------------------------------------------------
# Gradient against central differences of the oracle's own energy.
# ---------------------------------------------------------------------------------------------
def test_gradient_central_differences():
    wl = make_random(12, 20.0, 16.0, 24, 20, seed=13)
    W, H = wl.W, wl.H
    x, y, w, h = wl.arrays()
    E, a, _ = oracle.energy(W, H, x, y, w, h, wl.Mu, wl.Mp)
    gx, gy = oracle.grad(W, H, x, y, w, h, a)
    st = 1e-4
    for i in range(wl.n):
        for arr, g in ((x, gx), (y, gy)):
            old = arr[i]
            arr[i] = old + st
            Ep = _E(W, H, x, y, w, h, wl.Mu, wl.Mp)
            arr[i] = old - st
            Em = _E(W, H, x, y, w, h, wl.Mu, wl.Mp)
            arr[i] = old
            fd = (Ep - Em) / (2 * st)
            assert abs(fd - g[i]) <= 1e-7 * max(abs(g).max(), 1e-300)


# ---------------------------------------------------------------------------------------------
# Energy as a per-block bilinear form, and the point evaluators of psi (eq. psi) and xi
# (eq. ksi) against block quadrature and finite differences.
# ---------------------------------------------------------------------------------------------
def _gauss_box(x0, y0, w, h, k=24):
    t, wt = np.polynomial.legendre.leggauss(k)
    px = x0 + w / 2 * t
    py = y0 + h / 2 * t
    PX, PY = np.meshgrid(px, py, indexing="ij")
    WT = np.outer(wt, wt) * (w / 2) * (h / 2)
    return PX.ravel(), PY.ravel(), WT.ravel()


def test_block_potential_and_point_psi():
    wl = make_random(6, 10.0, 8.0, 12, 10, seed=17)
    W, H = wl.W, wl.H
    x, y, w, h = wl.arrays()
    E, a, _ = oracle.energy(W, H, x, y, w, h, wl.Mu, wl.Mp)
    N = oracle.block_potential(W, H, x, y, w, h, a)
    assert 0.5 * N.sum() == pytest.approx(E, rel=1e-13)
    for i in range(wl.n):
        px, py, wt = _gauss_box(x[i], y[i], w[i], h[i])
        psi, _, _ = oracle.point_field(W, H, a, px, py)
        assert np.sum(psi * wt) == pytest.approx(N[i], rel=1e-10, abs=1e-12 * np.abs(N).max())


def test_point_field_is_minus_gradient_and_integrates_to_force():
    wl = make_random(5, 12.0, 9.0, 14, 11, seed=19)
    W, H = wl.W, wl.H
    x, y, w, h = wl.arrays()
    E, a, _ = oracle.energy(W, H, x, y, w, h, wl.Mu, wl.Mp)
    rng = np.random.default_rng(0)
    px, py = rng.uniform(0, W, 20), rng.uniform(0, H, 20)
    psi, ex, ey = oracle.point_field(W, H, a, px, py)
    st = 1e-5
    pxp, _, _ = oracle.point_field(W, H, a, px + st, py)
    pxm, _, _ = oracle.point_field(W, H, a, px - st, py)
    pyp, _, _ = oracle.point_field(W, H, a, px, py + st)
    pym, _, _ = oracle.point_field(W, H, a, px, py - st)
    sc = max(np.abs(ex).max(), np.abs(ey).max())
    assert np.abs(-(pxp - pxm) / (2 * st) - ex).max() < 1e-7 * sc
    assert np.abs(-(pyp - pym) / (2 * st) - ey).max() < 1e-7 * sc
    gx, gy = oracle.grad(W, H, x, y, w, h, a)
    for i in range(wl.n):
        qx, qy, wt = _gauss_box(x[i], y[i], w[i], h[i])
        _, fx, fy = oracle.point_field(W, H, a, qx, qy)
        assert -np.sum(fx * wt) == pytest.approx(gx[i], abs=1e-10 * np.abs(gx).max())
        assert -np.sum(fy * wt) == pytest.approx(gy[i], abs=1e-10 * np.abs(gy).max())


# ---------------------------------------------------------------------------------------------
# Superposition across the oracle's internal block chunks, and agreement of its sampled
# routines with the full ones.
# ---------------------------------------------------------------------------------------------
def test_superposition_across_chunks_and_sampled_routines():
    wl = make_random(5000, 300.0, 200.0, 20, 16, seed=23, wmax=6.0, hmax=3.0)
    W, H = wl.W, wl.H
    x, y, w, h = wl.arrays()
    a, I = oracle.coeffs(W, H, x, y, w, h, wl.Mu, wl.Mp)
    k = 2900
    a1, _ = oracle.coeffs(W, H, x[:k], y[:k], w[:k], h[:k], wl.Mu, wl.Mp)
    a2, _ = oracle.coeffs(W, H, x[k:], y[k:], w[k:], h[k:], wl.Mu, wl.Mp)
    assert np.abs(a1 + a2 - a).max() < 1e-12 * np.abs(a).max()
    us = np.array([0, 1, 5, 19, 3, 0])
    ps = np.array([1, 0, 7, 15, 3, 0])
    asmp, Ismp = oracle.coeffs_sampled(W, H, x, y, w, h, us, ps)
    assert np.abs(asmp - a[us, ps]).max() <= 1e-13 * np.abs(a).max()
    assert np.abs(Ismp - I[us, ps]).max() <= 1e-13 * np.abs(I).max()
    idx = np.array([0, 17, 4999, 2048, 2047])
    sub = slice(0, 3000)
    gx, gy = oracle.grad(W, H, x[sub], y[sub], w[sub], h[sub], a)
    sx, sy = oracle.grad_sampled(W, H, x, y, w, h, a, idx[:2])
    assert np.array_equal(sx, gx[idx[:2]]) and np.array_equal(sy, gy[idx[:2]])


# ---------------------------------------------------------------------------------------------
# Stored values written by tests/golden/make_golden.py (oracle only): guard against silent
# changes of the oracle's arithmetic.
# ---------------------------------------------------------------------------------------------
def test_golden_oracle_cases_unchanged():
    import json
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "oracle_cases.json")
    for c in json.load(open(path))["cases"]:
        E, a, _ = oracle.energy(c["W"], c["H"], c["x"], c["y"], c["w"], c["h"], c["Mu"], c["Mp"])
        gx, gy = oracle.grad(c["W"], c["H"], c["x"], c["y"], c["w"], c["h"], a)
        assert E == pytest.approx(c["E"], rel=1e-14)
        assert np.allclose(a[:4, :4], c["a_corner"], rtol=1e-13, atol=1e-15 * np.abs(a).max())
        assert np.allclose(gx, c["gx"], rtol=1e-12, atol=1e-13 * np.abs(gx).max())
        assert np.allclose(gy, c["gy"], rtol=1e-12, atol=1e-13 * np.abs(gy).max())


# ---------------------------------------------------------------------------------------------
# The rank-one central-difference helper used by the large-workload GPU tests agrees with the
# oracle's gradient (and with brute-force central differences of the oracle's energy).
# ---------------------------------------------------------------------------------------------
def test_rank1_central_difference_helper():
    from tests.fd_rank1 import central_difference
    wl = make_random(400, 300.0, 200.0, 48, 40, seed=41, wmax=8.0, hmax=2.0)
    W, H = wl.W, wl.H
    x, y, w, h = wl.arrays()
    E, a, _ = oracle.energy(W, H, x, y, w, h, wl.Mu, wl.Mp)
    gx, gy = oracle.grad(W, H, x, y, w, h, a)
    idx = np.array([0, 7, 123, 399])
    fx, fy = central_difference(W, H, x, y, w, h, a, idx, 1e-3)
    sc = max(np.abs(gx).max(), np.abs(gy).max())
    assert np.abs(fx - gx[idx]).max() < 1e-6 * sc
    assert np.abs(fy - gy[idx]).max() < 1e-6 * sc
    # brute force for one block
    i = 7
    xp = x.copy(); xp[i] += 1e-3
    xm = x.copy(); xm[i] -= 1e-3
    bf = (_E(W, H, xp, y, w, h, wl.Mu, wl.Mp) - _E(W, H, xm, y, w, h, wl.Mu, wl.Mp)) / 2e-3
    assert abs(bf - fx[1]) < 1e-7 * sc


# ---------------------------------------------------------------------------------------------
# Bin scheme (Sec. III-D), the comparison path.
# ---------------------------------------------------------------------------------------------
def test_bin_density_hand_case():
    # W = H = 4, m = 4 (unit bins); one block over x in [0.5, 2], y in [1, 2]: half of bin (0, 1)
    # and all of bin (1, 1).  A second block overhangs the region's corner: only its inside part
    # [3.5, 4] x [3.5, 4] counts, a quarter of bin (3, 3).
    P = oracle.bin_density(4.0, 4.0, [1.25, 4.0], [1.5, 4.0], [1.5, 1.0], [1.0, 1.0], 4)
    ref = np.zeros((4, 4))
    ref[0, 1], ref[1, 1], ref[3, 3] = 0.5, 1.0, 0.25
    assert np.array_equal(P, ref)


def test_bin_density_exact_by_lattice_sampling():
    # Block edges on a lattice of 1/8 bin: sampling the lattice cell midpoints counts every cell
    # exactly, so the sampled bin areas are exact (an independent brute force).
    rng = np.random.default_rng(11)
    W, H, m, q = 6.0, 3.0, 6, 8
    wb, hb = W / m, H / m
    n = 40
    x0 = rng.integers(-4, m * q, n) * wb / q
    y0 = rng.integers(-4, m * q, n) * hb / q
    w = rng.integers(1, 3 * q, n) * wb / q
    h = rng.integers(1, 3 * q, n) * hb / q
    P = oracle.bin_density(W, H, x0 + w / 2, y0 + h / 2, w, h, m)
    xs = (np.arange(m * q) + 0.5) * wb / q
    ys = (np.arange(m * q) + 0.5) * hb / q
    cover = np.zeros((m * q, m * q))
    for i in range(n):
        inx = (xs > x0[i]) & (xs < x0[i] + w[i])
        iny = (ys > y0[i]) & (ys < y0[i] + h[i])
        cover += np.outer(inx, iny)
    ref = cover.reshape(m, q, m, q).sum(axis=(1, 3)) / (q * q)
    assert np.abs(P - ref).max() <= 1e-12


def test_bin_density_total_area():
    rng = np.random.default_rng(3)
    W, H, m, n = 10.0, 7.0, 9, 200
    x, y = rng.uniform(-1, W + 1, n), rng.uniform(-1, H + 1, n)
    w, h = rng.uniform(0.05, 3.0, n), rng.uniform(0.05, 2.0, n)
    P = oracle.bin_density(W, H, x, y, w, h, m)
    inside = (np.clip(np.minimum(x + w / 2, W) - np.maximum(x - w / 2, 0), 0, None)
              * np.clip(np.minimum(y + h / 2, H) - np.maximum(y - h / 2, 0), 0, None))
    assert P.sum() * (W / m) * (H / m) == pytest.approx(inside.sum(), rel=1e-13)


def _disa_from_dct(W, H, P, Mu, Mp):
    """Eqs. disa-a..d with the double sums taken by scipy's DCT-II."""
    m = P.shape[0]
    D = scipy.fft.dctn(P, type=2) / 4.0
    ref = np.zeros((Mu, Mp))
    uu, pp = np.meshgrid(np.arange(1, Mu), np.arange(1, Mp), indexing="ij")
    ref[1:, 1:] = (16 * W**2 * H**2 / (uu * pp * (uu**2 * H**2 + pp**2 * W**2) * PI**4)
                   * np.sin(uu * PI / (2 * m)) * np.sin(pp * PI / (2 * m)) * D[1:Mu, 1:Mp])
    pr, ur = np.arange(1, Mp), np.arange(1, Mu)
    ref[0, 1:] = 4 * H**2 / (pr**3 * PI**3 * m) * np.sin(pr * PI / (2 * m)) * D[0, 1:Mp]
    ref[1:, 0] = 4 * W**2 / (ur**3 * PI**3 * m) * np.sin(ur * PI / (2 * m)) * D[1:Mu, 0]
    return ref


@pytest.mark.parametrize("W,H,m,Mu,Mp", [(12.0, 5.0, 6, 6, 6), (3.0, 8.0, 10, 7, 10), (9.0, 9.0, 16, 16, 5)])
def test_bin_coeffs_match_dct2(W, H, m, Mu, Mp):
    P = np.random.default_rng(m).uniform(0.0, 2.0, (m, m))
    a = oracle.bin_coeffs(W, H, P, Mu, Mp)
    ref = _disa_from_dct(W, H, P, Mu, Mp)
    assert np.abs(a - ref).max() <= 1e-13 * np.abs(ref).max()
    assert a[0, 0] == 0.0


def test_bin_coeffs_equal_direct_sum_of_bin_blocks():
    # Whole-bin occupancy: the binned coefficients are the exact coefficients of the blocks.
    W, H, m = 8.0, 6.0, 8
    occ = np.random.default_rng(5).integers(0, 2, (m, m))
    l, j = np.nonzero(occ)
    xs, ys = (l + 0.5) * W / m, (j + 0.5) * H / m
    a_dir, _ = oracle.coeffs(W, H, xs, ys, np.full(len(xs), W / m), np.full(len(xs), H / m), m, m)
    P = oracle.bin_density(W, H, xs, ys, np.full(len(xs), W / m), np.full(len(xs), H / m), m)
    assert np.array_equal(P, occ.astype(float))
    a_bin = oracle.bin_coeffs(W, H, P, m, m)
    assert np.abs(a_bin - a_dir).max() <= 1e-13 * np.abs(a_dir).max()


@pytest.mark.parametrize("W,H,m,Mu,Mp", [(12.0, 5.0, 6, 6, 6), (4.0, 9.0, 9, 5, 9)])
def test_bin_field_matches_dct3_and_point_field(W, H, m, Mu, Mp):
    a = np.random.default_rng(m + Mu).normal(size=(Mu, Mp))
    psi, xix, xiy = oracle.bin_field(W, H, m, a)
    # psi by scipy's DCT-III: y_k = x_0 + 2 sum_{n>=1} x_n cos(pi n (2k+1)/(2m)) on each axis
    ap = np.zeros((m, m))
    ap[:Mu, :Mp] = a
    ap[1:, :] /= 2.0
    ap[:, 1:] /= 2.0
    ref = scipy.fft.dctn(ap, type=3)
    assert np.abs(psi - ref).max() <= 1e-13 * np.abs(ref).max()
    # psi and xi at the bin centres by the point evaluation of eqs. psi, ksi
    xc, yc = (np.arange(m) + 0.5) * W / m, (np.arange(m) + 0.5) * H / m
    X, Y = np.meshgrid(xc, yc, indexing="ij")
    ps, ex, ey = oracle.point_field(W, H, a, X.ravel(), Y.ravel())
    for got, want in ((psi, ps), (xix, ex), (xiy, ey)):
        assert np.abs(got.ravel() - want).max() <= 1e-13 * np.abs(want).max()


def test_bin_sampled_routines_match_full():
    rng = np.random.default_rng(21)
    W, H, m, n = 9.0, 4.0, 12, 120
    x, y = rng.uniform(-0.5, W + 0.5, n), rng.uniform(-0.5, H + 0.5, n)
    w, h = rng.uniform(0.05, 4.0, n), rng.uniform(0.05, 2.0, n)
    P = oracle.bin_density(W, H, x, y, w, h, m)
    ls, js = rng.integers(0, m, 30), rng.integers(0, m, 30)
    assert np.abs(oracle.bin_density_at(W, H, x, y, w, h, m, ls, js) - P[ls, js]).max() <= 1e-14
    a = oracle.bin_coeffs(W, H, P, m, 9)
    us, ps = rng.integers(0, m, 30), rng.integers(0, 9, 30)
    assert np.abs(oracle.bin_coeffs_at(W, H, P, us, ps) - a[us, ps]).max() <= 1e-14 * np.abs(a).max()


def test_bin_interp_exact_by_lattice_sampling():
    # Block values from bin values: with block edges on a lattice of 1/8 bin, summing the lattice
    # cells inside each block, each weighted by the value of the bin that holds it, is exact (an
    # independent brute force).  Distinct random fields for psi, xi_x and xi_y and a non-square
    # region catch a transposed or swapped field; the field sums carry the gradient's minus sign.
    rng = np.random.default_rng(17)
    W, H, m, q = 6.0, 3.0, 6, 8
    wb, hb = W / m, H / m
    n = 40
    x0 = rng.integers(-4, m * q, n) * wb / q
    y0 = rng.integers(-4, m * q, n) * hb / q
    w = rng.integers(1, 3 * q, n) * wb / q
    h = rng.integers(1, 3 * q, n) * hb / q
    fields = [rng.normal(size=(m, m)) for _ in range(3)]
    N, gx, gy = oracle.bin_interp(W, H, x0 + w / 2, y0 + h / 2, w, h, m, *fields)
    xs = (np.arange(m * q) + 0.5) * wb / q
    ys = (np.arange(m * q) + 0.5) * hb / q
    cell = (wb / q) * (hb / q)
    fine = [np.repeat(np.repeat(f, q, axis=0), q, axis=1) for f in fields]
    for i in range(n):
        inx = (xs > x0[i]) & (xs < x0[i] + w[i])
        iny = (ys > y0[i]) & (ys < y0[i] + h[i])
        mask = np.outer(inx, iny)
        ref = [cell * f[mask].sum() for f in fine]
        assert N[i] == pytest.approx(ref[0], abs=1e-12)
        assert gx[i] == pytest.approx(-ref[1], abs=1e-12)
        assert gy[i] == pytest.approx(-ref[2], abs=1e-12)


def test_bin_interp_is_the_adjoint_of_the_densities():
    # sum_i N_i = wb hb sum_lj P_lj psi_lj for any bin field, and a unit field gives every block
    # its area inside the region.
    rng = np.random.default_rng(23)
    W, H, m, n = 10.0, 7.0, 9, 150
    x, y = rng.uniform(-1, W + 1, n), rng.uniform(-1, H + 1, n)
    w, h = rng.uniform(0.05, 4.0, n), rng.uniform(0.05, 3.0, n)
    psi = rng.normal(size=(m, m))
    P = oracle.bin_density(W, H, x, y, w, h, m)
    N, gx, gy = oracle.bin_interp(W, H, x, y, w, h, m, psi)
    assert gx is None and gy is None
    assert N.sum() == pytest.approx((W / m) * (H / m) * (P * psi).sum(), rel=1e-12)
    N1, _, _ = oracle.bin_interp(W, H, x, y, w, h, m, np.ones((m, m)))
    inside = (np.clip(np.minimum(x + w / 2, W) - np.maximum(x - w / 2, 0), 0, None)
              * np.clip(np.minimum(y + h / 2, H) - np.maximum(y - h / 2, 0), 0, None))
    assert np.abs(N1 - inside).max() <= 1e-13 * inside.max()


def test_bin_scheme_block_values_converge_to_the_direct_ones():
    # For a smooth potential (few frequencies) the bin scheme's block potentials and gradients
    # approach the direct path's N_i and dE/dx_i, dE/dy_i as the bins shrink: the error of a partly
    # covered bin (value taken at its centre, not at the covered part's) is O(bin size) over O(bin
    # size) of the block's edge, so the relative error falls with the square of the bin size.  A
    # flipped sign of the field sums would leave an error near 2.
    rng = np.random.default_rng(29)
    W, H, n, M = 5.0, 4.0, 60, 4
    x, y = rng.uniform(0.5, W - 0.5, n), rng.uniform(0.5, H - 0.5, n)
    w, h = rng.uniform(0.2, 1.0, n), rng.uniform(0.2, 1.0, n)
    a = rng.normal(size=(M, M))
    N_dir = oracle.block_potential(W, H, x, y, w, h, a)
    gx_dir, gy_dir = oracle.grad(W, H, x, y, w, h, a)
    errs = []
    for m in (32, 128):
        N, gx, gy = oracle.bin_interp(W, H, x, y, w, h, m, *oracle.bin_field(W, H, m, a))
        errs.append(max(np.abs(N - N_dir).max() / np.abs(N_dir).max(),
                        np.abs(gx - gx_dir).max() / np.abs(gx_dir).max(),
                        np.abs(gy - gy_dir).max() / np.abs(gy_dir).max()))
    assert errs[0] < 2e-2 and errs[1] < 2e-3 and errs[1] < errs[0] / 8, errs


# ---------------------------------------------------------------------------------------------
# Raw block sums, their absolute counterparts and the closed-form prefactors (the quantities the
# tile-resolving parity metrics compare): S'_iu is w_u times the integral of cos(w_u t) over the
# block (the block width at u = 0), taken here by Gauss-Legendre quadrature rather than by the
# oracle's sine differences; R = sum_i S' T', Rabs = sum_i |S' T'|, and f R = a with the pinned a.
# ---------------------------------------------------------------------------------------------
def _quad_basis(c, s, L, M, nodes=64):
    t, wq = np.polynomial.legendre.leggauss(nodes)
    out = np.zeros((len(c), M))
    for i, (ci, si) in enumerate(zip(c, s)):
        pts = ci + 0.5 * si * t
        for k in range(M):
            wk = k * PI / L
            integ = 0.5 * si * np.sum(wq * np.cos(wk * pts))
            out[i, k] = integ * (wk if k > 0 else 1.0)
    return out


def test_raw_moments_and_absolute_sums_by_quadrature():
    wl = make_random(7, 30.0, 20.0, 11, 9, seed=71, wmax=6.0, hmax=5.0)
    Sx = _quad_basis(wl.x, wl.w, wl.W, wl.Mu)
    Ty = _quad_basis(wl.y, wl.h, wl.H, wl.Mp)
    Rq = Sx.T @ Ty
    Raq = np.abs(Sx).T @ np.abs(Ty)
    R = oracle.raw_moments(wl.W, wl.H, *wl.arrays(), wl.Mu, wl.Mp)
    assert np.allclose(R, Rq, rtol=0, atol=1e-12 * np.abs(Rq).max())
    us, ps = np.meshgrid(np.arange(wl.Mu), np.arange(wl.Mp), indexing="ij")
    us, ps = us.ravel(), ps.ravel()
    a_s, R_s, Ra_s = oracle.coeffs_sampled_full(wl.W, wl.H, *wl.arrays(), us, ps)
    assert np.allclose(R_s, Rq.ravel(), rtol=0, atol=1e-12 * np.abs(Rq).max())
    assert np.allclose(Ra_s, Raq.ravel(), rtol=1e-12, atol=1e-13 * Raq.max())
    a, _ = oracle.coeffs(wl.W, wl.H, *wl.arrays(), wl.Mu, wl.Mp)
    f = oracle.coef_factors(wl.W, wl.H, wl.Mu, wl.Mp)
    assert f[0, 0] == 0.0 and np.all(f.ravel()[1:] > 0)
    assert np.allclose(f * Rq, a, rtol=0, atol=1e-12 * np.abs(a).max())
    assert np.allclose(a_s, a.ravel(), rtol=1e-14, atol=0)
