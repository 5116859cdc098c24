"""Parity metrics that resolve every output tile (test infrastructure).

The coefficients fall like (u^2 + p^2)^-2 (Sec. III-A closed forms), so one relative norm over the
whole coefficient array, the energy or the gradient is dominated by the lowest frequencies: a tile
of 256 x 256 frequencies beyond the first one could be wrong or missing and the norm would move by
less than 1e-4.  The metrics here give every part of the output its own weight:

* coefficients: the raw block sums R_up = sum_i S'_iu T'_ip = a_up / f_up (f_up the prefactor of
  the closed forms, taken from the oracle), whose magnitude does not fall with (u, p), compared per
  tile of TILE x TILE frequencies (finer than every output tile of the kernels);
* gradients and evaluation rows: inputs whose contracted operand is ~N(0, 1) over the whole
  frequency plane ("flat" coefficients, any coefficients being valid inputs of these linear maps),
  compared per tile of ROW_TILE blocks (or points);
* full-size samples: each sampled coefficient on its own, scaled by f_up sum_i |S'_iu T'_ip| (the
  magnitude that bounds the rounding of its sum), with samples in every output tile.

Only the seeded inputs come from here; every expected value comes from the oracle.
"""
from __future__ import annotations

import numpy as np

TILE = 64          # coefficient tiles (u x p) of the per-tile metric
ROW_TILE = 256     # block (or point) tiles of the per-tile metric of per-block outputs
KERNEL_TILE = 256  # output tile of the bf16 contractions: full-size samples cover each one


def rel(a, b):
    """Relative error ||a - b|| / ||b|| (0-norm-safe)."""
    a = np.ravel(np.asarray(a, dtype=np.float64))
    b = np.ravel(np.asarray(b, dtype=np.float64))
    nb = float(np.linalg.norm(b))
    return float(np.linalg.norm(a - b)) / (nb if nb > 0 else 1.0)


def raw_from_coeffs(a, f):
    """R = a / f where f != 0 (the (0, 0) entry, whose prefactor vanishes, is set to 0)."""
    a = np.asarray(a, dtype=np.float64)
    out = np.zeros_like(a)
    nz = f != 0
    out[nz] = a[nz] / f[nz]
    return out


def tile_rel_max(A, B, tu=TILE, tp=TILE):
    """Largest relative error over the tiles of a 2-D array: max_t ||A_t - B_t|| / ||B_t||, and the
    worst tile's origin.  Tiles whose reference is exactly zero are judged by their absolute error
    against the largest tile norm."""
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    Mu, Mp = B.shape
    norms = {}
    for u0 in range(0, Mu, tu):
        for p0 in range(0, Mp, tp):
            norms[(u0, p0)] = float(np.linalg.norm(B[u0:u0 + tu, p0:p0 + tp]))
    big = max(norms.values()) if norms else 0.0
    worst, where = 0.0, None
    for (u0, p0), nb in norms.items():
        d = float(np.linalg.norm(A[u0:u0 + tu, p0:p0 + tp] - B[u0:u0 + tu, p0:p0 + tp]))
        den = nb if nb > 0 else (big if big > 0 else 1.0)
        e = d / den
        if e > worst or where is None:
            worst, where = e, (u0, p0)
    return worst, where


def coeff_errors(a, R_ref, f):
    """Errors of GPU coefficients a against the oracle's raw sums R_ref: the whole flat-spectrum
    relative error and the worst TILE x TILE tile."""
    R = raw_from_coeffs(a, f)
    Rr = np.where(f != 0, R_ref, 0.0)
    t, where = tile_rel_max(R, Rr)
    return {"flat": rel(R, Rr), "flat_tile": t, "flat_tile_at": where}


def row_tile_rel_max(g, g_ref, tile=ROW_TILE):
    """Largest relative error over tiles of `tile` consecutive rows of per-block outputs (g may be
    [n] or [n, k]); zero-reference tiles are judged against the largest tile norm."""
    g = np.asarray(g, dtype=np.float64).reshape(len(g_ref), -1)
    g_ref = np.asarray(g_ref, dtype=np.float64).reshape(len(g_ref), -1)
    n = g_ref.shape[0]
    if n == 0:
        return 0.0
    norms = [float(np.linalg.norm(g_ref[i:i + tile])) for i in range(0, n, tile)]
    big = max(norms)
    worst = 0.0
    for k, i in enumerate(range(0, n, tile)):
        den = norms[k] if norms[k] > 0 else (big if big > 0 else 1.0)
        worst = max(worst, float(np.linalg.norm(g[i:i + tile] - g_ref[i:i + tile])) / den)
    return worst


def _freq_scale(M, L):
    k = np.arange(M, dtype=np.float64)
    return np.where(k > 0, k * np.pi / L, 1.0)


def flat_field_coeffs(W, H, Mu, Mp, seed):
    """Two coefficient sets for the gradient: with a_x the operand a_up / vt_p of gx is ~N(0, 1),
    with a_y the operand a_up / wt_u of gy is ~N(0, 1) (wt_u = u pi / W, 1 at u = 0; vt likewise)."""
    rng = np.random.default_rng(seed)
    nx = rng.normal(size=(Mu, Mp))
    ny = rng.normal(size=(Mu, Mp))
    a_x = nx * _freq_scale(Mp, H)[None, :]
    a_y = ny * _freq_scale(Mu, W)[:, None]
    return np.ascontiguousarray(a_x), np.ascontiguousarray(a_y)


def flat_point_coeffs(Mu, Mp, seed):
    """Coefficients ~N(0, 1): the operand of the point potential and field is a itself."""
    return np.random.default_rng(seed).normal(size=(Mu, Mp))


def flat_potential_coeffs(W, H, Mu, Mp, seed):
    """Coefficients whose block-potential operand a_up / (wt_u vt_p) is ~N(0, 1)."""
    rng = np.random.default_rng(seed)
    return rng.normal(size=(Mu, Mp)) * _freq_scale(Mu, W)[:, None] * _freq_scale(Mp, H)[None, :]


def samples_per_tile(Mu, Mp, per_tile, seed, tile=KERNEL_TILE):
    """(us, ps): `per_tile` seeded frequency pairs in every tile x tile output tile (fewer where a
    ragged tile holds fewer pairs), never (0, 0)."""
    rng = np.random.default_rng(seed)
    us, ps = [], []
    for u0 in range(0, Mu, tile):
        for p0 in range(0, Mp, tile):
            nu, np_ = min(tile, Mu - u0), min(tile, Mp - p0)
            k = min(per_tile, nu * np_ - (1 if u0 == 0 and p0 == 0 else 0))
            if k <= 0:
                continue
            flat = rng.choice(nu * np_, size=min(nu * np_, k + 1), replace=False)
            got = 0
            for q in flat:
                u, p = u0 + int(q) // np_, p0 + int(q) % np_
                if u == 0 and p == 0:
                    continue
                us.append(u)
                ps.append(p)
                got += 1
                if got == k:
                    break
    return np.array(us, dtype=np.int64), np.array(ps, dtype=np.int64)


def scaled_sample_errors(a_samples, a_ref, f_samples, Rabs):
    """Per-sample errors |a - a*| / (|f_up| sum_i |S'_iu T'_ip|)."""
    den = np.abs(f_samples) * Rabs
    den = np.where(den > 0, den, 1.0)
    return np.abs(np.asarray(a_samples) - np.asarray(a_ref)) / den


def tile_max_of_samples(errs, us, ps, tile=KERNEL_TILE):
    """The largest sample error of every output tile that holds samples: {(u0, p0): err}."""
    out = {}
    for e, u, p in zip(errs, us, ps):
        key = (int(u) // tile * tile, int(p) // tile * tile)
        out[key] = max(out.get(key, 0.0), float(e))
    return out
