"""Exact central energy differences for one moved block (test helper, numpy FP64).

E = 1/2 sum_up s_up A_up^2 with A_up = sum_i X_iu Y_ip (the block moments of the truncated series,
Sec. III-A; s_up the spectral scale of the coefficient closed forms, s_00 = 0).  Moving block i by
+-h in x changes only its x integrals, A -> A + dX+- (x) Y_i, so

    E(x_i + h) - E(x_i - h) = sum_up a_up (d+ - d-)_up + 1/2 sum_up s_up ((d+)^2 - (d-)^2)_up,

with a = s A the coefficients and d+- = (X_i(x_i +- h) - X_i(x_i)) (x) Y_i.  The change of the sine
integral is written without cancellation:
    X_u(x + t) - X_u(x) = [2 cos(w_u e+ + w_u t/2) - 2 cos(w_u e- + w_u t/2)] sin(w_u t / 2) / w_u.
The central difference (E(x+h) - E(x-h)) / 2h is then exact up to its O(h^2) truncation, at any n,
given the coefficients a of the same blocks.
"""
import numpy as np


def _scale(W, H, Mu, Mp):
    wu = np.arange(Mu) * np.pi / W
    vp = np.arange(Mp) * np.pi / H
    eps = np.outer(np.where(np.arange(Mu) > 0, 2.0, 1.0), np.where(np.arange(Mp) > 0, 2.0, 1.0))
    with np.errstate(divide="ignore"):
        s = eps / (W * H * (wu[:, None] ** 2 + vp[None, :] ** 2))
    s[0, 0] = 0.0
    return s


def _integral(c, sz, L, M):
    k = np.arange(M)
    w = k * np.pi / L
    out = np.empty(M)
    out[0] = sz
    out[1:] = 2.0 * np.cos(w[1:] * c) * np.sin(w[1:] * sz / 2.0) / w[1:]
    return out


def _shift(c, sz, L, M, t):
    """X_k(c + t) - X_k(c) for k < M (0 for k = 0)."""
    k = np.arange(M)
    w = k * np.pi / L
    out = np.zeros(M)
    ww = w[1:]
    ep, em = c + sz / 2.0, c - sz / 2.0
    out[1:] = (2.0 * np.cos(ww * ep + ww * t / 2.0) - 2.0 * np.cos(ww * em + ww * t / 2.0)) * np.sin(ww * t / 2.0) / ww
    return out


def central_difference(W, H, x, y, w, h, a, idx, step):
    """(dE/dx_i, dE/dy_i) by exact central differences with step `step` for the blocks idx."""
    a = np.asarray(a, dtype=np.float64)
    Mu, Mp = a.shape
    s = _scale(W, H, Mu, Mp)
    gx = np.empty(len(idx))
    gy = np.empty(len(idx))
    for n_, i in enumerate(idx):
        Xi = _integral(x[i], w[i], W, Mu)
        Yi = _integral(y[i], h[i], H, Mp)
        dp, dm = _shift(x[i], w[i], W, Mu, step), _shift(x[i], w[i], W, Mu, -step)
        Dp, Dm = np.outer(dp, Yi), np.outer(dm, Yi)
        gx[n_] = (np.sum(a * (Dp - Dm)) + 0.5 * np.sum(s * (Dp * Dp - Dm * Dm))) / (2.0 * step)
        ep, em = _shift(y[i], h[i], H, Mp, step), _shift(y[i], h[i], H, Mp, -step)
        Ep, Em = np.outer(Xi, ep), np.outer(Xi, em)
        gy[n_] = (np.sum(a * (Ep - Em)) + 0.5 * np.sum(s * (Ep * Ep - Em * Em))) / (2.0 * step)
    return gx, gy
