"""GPU-versus-oracle comparison shared by the GPU parity tests (test infrastructure).

For one workload and one precision (and basis mode) it runs pp_energy and pp_field through the
binding, and pp_field again on two sets of flat-spectrum coefficients (one makes the gx operand
~N(0, 1) over the whole frequency plane, the other the gy operand), and compares with the FP64
oracle on the same seeded inputs:

* coefficients: ||a - a*|| / ||a*||, and the raw block sums a / f against the oracle's, over the
  whole array and per 64 x 64 tile (tests/parity.py);
* energy: |E - E*| / |E*|;
* gradient of the run's own coefficients (against the oracle's gradient of the oracle's
  coefficients): the norm over all blocks and the worst tile of 256 blocks;
* gradient of the flat coefficients: gx and gy each over all blocks and per 256-block tile.

Every metric of a check is held to the same bar.  Expected values come from the oracle only.
"""
from __future__ import annotations

import sys

import numpy as np

import oracle
from tests import parity

DEV = "cuda:0"


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def dev(*arrs):
    import torch
    return [torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device=DEV) for a in arrs]


class OracleRef:
    """The oracle's results for one workload (computed once, shared by several precisions)."""

    def __init__(self, wl, grad_sample=None, flat_seed=17):
        self.wl = wl
        E, a, _ = oracle.energy(wl.W, wl.H, *wl.arrays(), wl.Mu, wl.Mp)
        self.E, self.a = E, a
        self.f = oracle.coef_factors(wl.W, wl.H, wl.Mu, wl.Mp)
        self.R = parity.raw_from_coeffs(a, self.f)
        if grad_sample is None:
            self.idx = np.arange(wl.n)
        else:
            self.idx = np.sort(np.random.default_rng(0).choice(wl.n, grad_sample, replace=False))
        self.a_x, self.a_y = parity.flat_field_coeffs(wl.W, wl.H, wl.Mu, wl.Mp, flat_seed)
        arrs = wl.arrays()
        if grad_sample is None:
            self.gx, self.gy = oracle.grad(wl.W, wl.H, *arrs, a)
            self.gx_flat, _ = oracle.grad(wl.W, wl.H, *arrs, self.a_x)
            _, self.gy_flat = oracle.grad(wl.W, wl.H, *arrs, self.a_y)
        else:
            self.gx, self.gy = oracle.grad_sampled(wl.W, wl.H, *arrs, a, self.idx)
            self.gx_flat, _ = oracle.grad_sampled(wl.W, wl.H, *arrs, self.a_x, self.idx)
            _, self.gy_flat = oracle.grad_sampled(wl.W, wl.H, *arrs, self.a_y, self.idx)


def run_gpu(wl, prec, basis="recompute", ref=None):
    """(E, a, gx, gy, gx_flat, gy_flat) of the library for workload wl (the flat gradients only if
    ref is given: its flat coefficients)."""
    import torch

    import paper_2307_12041_amd as pp
    x, y, w, h = dev(*wl.arrays())
    ws = torch.empty(max(pp.workspace_size(wl.W, wl.H, wl.n, wl.Mu, wl.Mp, precision=prec, basis=basis), 1),
                     dtype=torch.uint8, device=DEV)
    kw = dict(W=wl.W, H=wl.H, precision=prec, basis=basis, workspace=ws)
    E, a = pp.energy(x, y, w, h, Mu=wl.Mu, Mp=wl.Mp, **kw)
    gx, gy = pp.field(x, y, w, h, a, **kw)
    out = [float(E.cpu()), a.cpu().numpy(), gx.cpu().numpy(), gy.cpu().numpy()]
    if ref is not None:
        ax, ay = dev(ref.a_x, ref.a_y)
        gxf, _ = pp.field(x, y, w, h, ax, **kw)
        _, gyf = pp.field(x, y, w, h, ay, **kw)
        out += [gxf.cpu().numpy(), gyf.cpu().numpy()]
    torch.cuda.synchronize()
    return out


def errors(ref, E, a, gx, gy, gx_flat=None, gy_flat=None):
    """All metrics of one run against the oracle reference."""
    i = ref.idx
    ce = parity.coeff_errors(a, ref.R, ref.f)
    g = np.stack([gx[i], gy[i]], axis=1)
    go = np.stack([ref.gx, ref.gy], axis=1)
    out = {"a": parity.rel(a, ref.a), "a_flat": ce["flat"], "a_flat_tile": ce["flat_tile"],
           "E": abs(E - ref.E) / (abs(ref.E) if ref.E else 1.0),
           "g": parity.rel(g, go), "g_tile": parity.row_tile_rel_max(g, go)}
    if gx_flat is not None:
        out["gx_flat"] = parity.rel(gx_flat[i], ref.gx_flat)
        out["gy_flat"] = parity.rel(gy_flat[i], ref.gy_flat)
        out["gx_flat_tile"] = parity.row_tile_rel_max(gx_flat[i], ref.gx_flat)
        out["gy_flat_tile"] = parity.row_tile_rel_max(gy_flat[i], ref.gy_flat)
    out["_worst_a_tile"] = ce["flat_tile_at"]
    return out


def fmt(errs):
    return " ".join(f"{k}={v:.2e}" for k, v in errs.items() if not k.startswith("_"))


def check(wl, prec, tol, basis="recompute", ref=None, grad_sample=None, label="parity"):
    """Run and compare; every metric must be <= tol.  Returns (errors, gpu outputs)."""
    say(f"[{label}] {wl.name} n={wl.n} Mu={wl.Mu} Mp={wl.Mp} prec={prec} basis={basis}")
    if ref is None:
        ref = OracleRef(wl, grad_sample=grad_sample)
    outs = run_gpu(wl, prec, basis, ref)
    errs = errors(ref, *outs)
    say(f"   {fmt(errs)}")
    bad = {k: v for k, v in errs.items() if not k.startswith("_") and not v <= tol}
    assert not bad, (prec, basis, bad, errs["_worst_a_tile"])
    return errs, outs
