"""Invariants of the exact solution re-run through the C ABI at every precision and basis mode
(tile-edge and indexing checks that need no oracle): blocks tiling the region give a = 0, E = 0,
g = 0 at any truncation; a block centred in the region has zero odd-index coefficients and zero
gradient; mirroring x -> W - x leaves E unchanged, negates gx and keeps gy; E is non-negative and
grows with the truncation.  Sizes are odd and unequal (Mu != Mp, neither a multiple of a tile,
n not a multiple of a chunk)."""
import sys

import numpy as np
import pytest

from tests.fd_rank1 import _scale
from workloads import make_random

torch = pytest.importorskip("torch")
pp = pytest.importorskip("paper_2307_12041_amd")

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
TOL = {"fp64": 1e-10, "fp32": 1e-5, "bf16x3": 1e-3, "bf16": 3e-2}
MODES = [("fp64", "recompute"), ("fp32", "recompute"), ("bf16x3", "recompute"), ("bf16", "recompute"),
         ("bf16x3", "store"), ("bf16", "store")]


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def dev(*arrs):
    return [torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device=DEV) for a in arrs]


def run(x, y, w, h, W, H, Mu, Mp, prec, basis):
    kw = dict(W=W, H=H, precision=prec, basis=basis)
    ws = torch.empty(pp.workspace_size(W, H, x.numel(), Mu, Mp, precision=prec, basis=basis), dtype=torch.uint8,
                     device=DEV)
    E, a = pp.energy(x, y, w, h, Mu=Mu, Mp=Mp, workspace=ws, **kw)
    gx, gy = pp.field(x, y, w, h, a, workspace=ws, **kw)
    torch.cuda.synchronize()
    return float(E.cpu()), a.cpu().numpy(), gx.cpu().numpy(), gy.cpu().numpy()


def term_bounds(sz, L, M):
    """Largest magnitudes of the block integral Xbar_ik = 2 cos(w_k c) sin(w_k sz/2) / w_k (|sz| for
    k = 0) and of K_ik = -2 sin(w_k c) sin(w_k sz/2): 2 / w_k and 2.  Every precision's rounding
    error of a basis value is a fraction of these, also where the value itself cancels to zero."""
    wk = np.arange(1, M) * np.pi / L
    xb = np.empty((len(sz), M))
    xb[:, 0] = np.abs(sz)
    xb[:, 1:] = 2.0 / wk
    kd = np.full((len(sz), M), 2.0)
    kd[:, 0] = 0.0
    return xb, kd


@pytest.mark.parametrize("prec,basis", MODES)
def test_tiling_gives_zero(prec, basis):
    # 13 x 7 blocks of 2 x 3 tile the 26 x 21 region exactly, so every moment A_up with (u, p) !=
    # (0, 0) cancels to zero.  The residue is bounded against the largest magnitudes of its terms
    # (term_bounds: m_x, m_y, m_K, m_L), at a tenth of each precision's parity bar:
    # |a_up| <= t s_up sum_i m_x,iu m_y,ip, E <= t^2 (1/2) sum (s M)^2 / s, and the gradient by the
    # same bound carried through m_K m_y (gx) or m_x m_L (gy).
    W, H, Mu, Mp = 26.0, 21.0, 301, 259
    xs, ys = np.meshgrid(np.arange(13) * 2 + 1.0, np.arange(7) * 3 + 1.5, indexing="ij")
    x, y = xs.ravel(), ys.ravel()
    n = x.size
    w, h = np.full(n, 2.0), np.full(n, 3.0)
    E0, a0, gx0, gy0 = run(*dev(x, y, w, h), W, H, Mu, Mp, prec, basis)
    xa, ka = term_bounds(w, W, Mu)
    ya, la = term_bounds(h, H, Mp)
    s = _scale(W, H, Mu, Mp)
    bound = s * (xa.T @ ya)                              # s_up sum_i m_x,iu m_y,ip
    tol = TOL[prec] / 10
    nz = s > 0
    say(f"[invariant] tiling {prec}/{basis}: max |a| / bound = {np.max(np.abs(a0)[nz] / bound[nz]):.2e}, E = {E0:.2e}")
    assert np.all(np.abs(a0) <= tol * bound + 1e-300)
    assert abs(E0) <= tol * tol * 0.5 * np.sum(bound[nz] ** 2 / s[nz])
    assert np.all(np.abs(gx0) <= tol * np.sum(ka * (ya @ bound.T), axis=1))
    assert np.all(np.abs(gy0) <= tol * np.sum(la * (xa @ bound), axis=1))


@pytest.mark.parametrize("prec,basis", MODES)
def test_centred_block_and_mirror(prec, basis):
    W, H, Mu, Mp = 40.0, 30.0, 67, 45
    tol = TOL[prec]
    # one block centred in the region: odd u or odd p coefficients vanish, and so does its gradient
    E, a, gx, gy = run(*dev([W / 2], [H / 2], [7.0], [4.5]), W, H, Mu, Mp, prec, basis)
    _, _, gxo, gyo = run(*dev([W / 2 + 3.0], [H / 2 - 2.0], [7.0], [4.5]), W, H, Mu, Mp, prec, basis)
    amax = np.abs(a).max()
    assert np.abs(a[1::2, :]).max() <= tol * amax and np.abs(a[:, 1::2]).max() <= tol * amax
    assert max(abs(gx[0]), abs(gy[0])) <= tol * max(abs(gxo[0]), abs(gyo[0]))
    # mirror images: x -> W - x keeps E, negates gx, keeps gy (and likewise in y)
    wl = make_random(517, W, H, Mu, Mp, seed=61, wmax=5.0, hmax=3.0)
    x, y, w, h = dev(*wl.arrays())
    E0, _, gx0, gy0 = run(x, y, w, h, W, H, Mu, Mp, prec, basis)
    E1, _, gx1, gy1 = run(W - x, y, w, h, W, H, Mu, Mp, prec, basis)
    E2, _, gx2, gy2 = run(x, H - y, w, h, W, H, Mu, Mp, prec, basis)
    g = max(np.abs(gx0).max(), np.abs(gy0).max())
    say(f"[invariant] mirror {prec}/{basis}: dE={abs(E1 - E0) / E0:.2e}, {abs(E2 - E0) / E0:.2e}")
    assert abs(E1 - E0) <= tol * E0 and abs(E2 - E0) <= tol * E0
    assert np.abs(gx1 + gx0).max() <= tol * g and np.abs(gy1 - gy0).max() <= tol * g
    assert np.abs(gx2 - gx0).max() <= tol * g and np.abs(gy2 + gy0).max() <= tol * g


@pytest.mark.parametrize("prec,basis", MODES)
def test_energy_non_negative_and_growing_with_truncation(prec, basis):
    W, H = 50.0, 35.0
    wl = make_random(333, W, H, 8, 8, seed=67, wmax=6.0, hmax=2.0)
    x, y, w, h = dev(*wl.arrays())
    Es = [run(x, y, w, h, W, H, Mu, Mp, prec, basis)[0] for Mu, Mp in ((5, 7), (5, 70), (90, 70), (257, 300))]
    say(f"[invariant] energies {prec}/{basis}: " + " ".join(f"{e:.6e}" for e in Es))
    tol = TOL[prec]
    assert Es[0] > 0.0
    for lo, hi in zip(Es, Es[1:]):
        assert hi >= lo * (1.0 - tol)
