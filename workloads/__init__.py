"""Seeded synthetic placement inputs shared by the tests, the benchmark and the oracle.

This module draws block rectangles only.  It holds none of the method's arithmetic
(no basis functions, no coefficients, no energy), so that the GPU library and the FP64
oracle can both be fed from it without sharing any computation.

Every workload is a rectangle region [0, W] x [0, H] (Sec. II-A of arXiv 2307.12041)
with n blocks given by centre (x_i, y_i) and size (w_i, h_i), plus the truncation
Mu x Mp of the cosine series (u in [0, Mu), p in [0, Mp)).

Draw order inside one workload (numpy ``default_rng(seed)``):
cell widths, macro widths, macro heights, cluster centres, cluster labels, centres
(x then y), then the clamp that keeps every block inside the region.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

__all__ = ["Workload", "CONFIGS", "make_config", "make_random", "jitter", "clamp_into_region"]


@dataclass
class Workload:
    name: str
    W: float
    H: float
    Mu: int
    Mp: int
    x: np.ndarray
    y: np.ndarray
    w: np.ndarray
    h: np.ndarray
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.x.shape[0])

    @property
    def pairs(self) -> int:
        """Work units of one evaluation: one (block, u, p) triple each."""
        return self.n * self.Mu * self.Mp

    def arrays(self):
        return self.x, self.y, self.w, self.h


# The five workloads.  Sizes, regions, truncations and size/position distributions follow the
# placement benchmarks the paper evaluates on (211K-2.5M blocks, cells of unit height mixed
# with large macros), scaled out to 10M blocks.  Names say what each one is.
CONFIGS = {
    1: dict(name="uniform_1k_1024sq_M64", n_cells=1000, cell_w=(1.0, 4.0), n_macros=0,
            macro_side=None, W=1024.0, H=1024.0, Mu=64, Mp=64, clusters=0, cluster_frac=0.0,
            sigma=None),
    2: dict(name="cells200k_macros50_8192sq_M512", n_cells=200_000, cell_w=(1.0, 8.0), n_macros=50,
            macro_side=(20.0, 200.0), W=8192.0, H=8192.0, Mu=512, Mp=512, clusters=0,
            cluster_frac=0.0, sigma=None),
    3: dict(name="cells1m_16clusters_16384sq_M1024", n_cells=1_000_000, cell_w=(1.0, 8.0), n_macros=0,
            macro_side=None, W=16384.0, H=16384.0, Mu=1024, Mp=1024, clusters=16, cluster_frac=1.0,
            sigma=800.0),
    4: dict(name="cells2m_macros500_16384sq_M2048", n_cells=2_000_000, cell_w=(1.0, 8.0), n_macros=500,
            macro_side=(50.0, 400.0), W=16384.0, H=16384.0, Mu=2048, Mp=2048, clusters=0,
            cluster_frac=0.0, sigma=None),
    5: dict(name="cells10m_64clusters_32768x16384_M4096x2048", n_cells=10_000_000, cell_w=(1.0, 8.0),
            n_macros=0, macro_side=None, W=32768.0, H=16384.0, Mu=4096, Mp=2048, clusters=64,
            cluster_frac=0.7, sigma=800.0),
}


def clamp_into_region(x, y, w, h, W, H):
    """Clamp centres so that every block lies inside [0, W] x [0, H] (blocks wider than the
    region are centred)."""
    lox = np.minimum(w / 2.0, W / 2.0)
    loy = np.minimum(h / 2.0, H / 2.0)
    x = np.clip(x, lox, W - lox)
    y = np.clip(y, loy, H - loy)
    return x, y


def _draw(spec: dict, seed: int, n_cells: int | None = None) -> Workload:
    rng = np.random.default_rng(seed)
    W, H = float(spec["W"]), float(spec["H"])
    nc = spec["n_cells"] if n_cells is None else int(n_cells)
    nm = spec["n_macros"]
    # 1. cell widths (continuous uniform), unit height
    cw = rng.uniform(spec["cell_w"][0], spec["cell_w"][1], size=nc)
    ch = np.ones(nc)
    # 2./3. macro widths and heights, independent
    if nm:
        lo, hi = spec["macro_side"]
        mw = rng.uniform(lo, hi, size=nm)
        mh = rng.uniform(lo, hi, size=nm)
    else:
        mw = np.empty(0)
        mh = np.empty(0)
    w = np.concatenate([cw, mw])
    h = np.concatenate([ch, mh])
    n = w.shape[0]
    # 4./5. cluster centres (uniform in the region) and equal-weight labels
    k = spec["clusters"]
    if k:
        cc = np.stack([rng.uniform(0.0, W, size=k), rng.uniform(0.0, H, size=k)], axis=1)
        n_cl = int(round(spec["cluster_frac"] * n))
        labels = rng.integers(0, k, size=n_cl)
    else:
        cc = None
        n_cl = 0
        labels = None
    # 6. centres: the first n_cl blocks around their cluster centre, the rest uniform
    x = rng.uniform(0.0, W, size=n)
    y = rng.uniform(0.0, H, size=n)
    if n_cl:
        s = spec["sigma"]
        x[:n_cl] = cc[labels, 0] + s * rng.standard_normal(n_cl)
        y[:n_cl] = cc[labels, 1] + s * rng.standard_normal(n_cl)
    x, y = clamp_into_region(x, y, w, h, W, H)
    return Workload(spec["name"], W, H, int(spec["Mu"]), int(spec["Mp"]),
                    np.ascontiguousarray(x), np.ascontiguousarray(y),
                    np.ascontiguousarray(w), np.ascontiguousarray(h),
                    meta=dict(seed=seed, n_cells=nc, n_macros=nm))


def make_config(k: int, seed: int | None = None, n_cells: int | None = None) -> Workload:
    """Workload ``k`` (1..5).  ``seed`` defaults to ``k``; ``n_cells`` overrides the cell count
    (used only to build scaled-down variants with the same distributions)."""
    spec = CONFIGS[k]
    return _draw(spec, k if seed is None else seed, n_cells)


def make_random(n: int, W: float, H: float, Mu: int, Mp: int, seed: int,
                wmax: float | None = None, hmax: float | None = None,
                inside: bool = True) -> Workload:
    """Small generic problem for tests: sizes uniform in (0.02, wmax] x (0.02, hmax], centres
    uniform.  With ``inside`` the blocks are clamped into the region."""
    rng = np.random.default_rng(seed)
    wmax = W / 8.0 if wmax is None else wmax
    hmax = H / 8.0 if hmax is None else hmax
    w = rng.uniform(0.02, wmax, size=n)
    h = rng.uniform(0.02, hmax, size=n)
    x = rng.uniform(0.0, W, size=n)
    y = rng.uniform(0.0, H, size=n)
    if inside:
        x, y = clamp_into_region(x, y, w, h, W, H)
    return Workload(f"random_n{n}_s{seed}", float(W), float(H), int(Mu), int(Mp), x, y, w, h,
                    meta=dict(seed=seed))


def jitter(wl: Workload, it: int, sigma: float = 1.0, seed: int = 1000) -> Workload:
    """Positions of iteration ``it`` of the repeated-evaluation workload: i.i.d. N(0, sigma^2)
    per coordinate added to the base positions, then clamped into the region."""
    rng = np.random.default_rng([seed, it])
    x = wl.x + sigma * rng.standard_normal(wl.n)
    y = wl.y + sigma * rng.standard_normal(wl.n)
    x, y = clamp_into_region(x, y, wl.w, wl.h, wl.W, wl.H)
    return Workload(f"{wl.name}_it{it}", wl.W, wl.H, wl.Mu, wl.Mp, x, y, wl.w, wl.h,
                    meta=dict(wl.meta, jitter_iteration=it))
