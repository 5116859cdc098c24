"""FP64 CPU oracle for the truncated cosine-series Poisson solution (arXiv 2307.12041, Sec. III-A).

TEST INFRASTRUCTURE ONLY.  The oracle is the independent checker of the GPU library: only the
tests, the smoke check and the CPU-baseline leg of the benchmark may import it.  The GPU library
never calls it and the two share no code.

The arithmetic lives in ``pp_oracle.c`` (plain C, double precision, long-double block sums,
OpenMP over independent outputs).  This module only builds and loads it and marshals numpy
arrays.  See the C file's header for the formulas and the passages of the paper they follow.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pp_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)
_lp = ctypes.POINTER(ctypes.c_int64)


def build(force: bool = True) -> str:
    """Compile the oracle into ``oracle/liboracle.so`` with gcc (-O2, OpenMP)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp"
        subprocess.run(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", _SRC, "-o", tmp, "-lm"],
                       check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    override = os.environ.get("PP_ORACLE_LIB")   # a deliberately broken copy, for mutation tests
    if override:
        lib = ctypes.CDLL(override)
    else:
        if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(_LIB_PATH)
    d, i64, i32 = ctypes.c_double, ctypes.c_int64, ctypes.c_int
    lib.oracle_coeffs.argtypes = [d, d, i64, _dp, _dp, _dp, _dp, i32, i32, _dp, _dp]
    lib.oracle_energy.argtypes = [d, d, i64, _dp, _dp, _dp, _dp, i32, i32, _dp, _dp, _dp]
    lib.oracle_grad.argtypes = [d, d, i64, _dp, _dp, _dp, _dp, i32, i32, _dp, _dp, _dp]
    lib.oracle_grad_sampled.argtypes = [d, d, _dp, _dp, _dp, _dp, i32, i32, _dp, i64, _lp, _dp, _dp]
    lib.oracle_coeffs_sampled.argtypes = [d, d, i64, _dp, _dp, _dp, _dp, i32, _ip, _ip, _dp, _dp]
    lib.oracle_coeffs_sampled_full.argtypes = [d, d, i64, _dp, _dp, _dp, _dp, i32, _ip, _ip, _dp, _dp, _dp, _dp]
    lib.oracle_raw_moments.argtypes = [d, d, i64, _dp, _dp, _dp, _dp, i32, i32, _dp]
    lib.oracle_coef_factors.argtypes = [d, d, i32, i32, _dp]
    lib.oracle_point_field.argtypes = [d, d, i32, i32, _dp, i64, _dp, _dp, _dp, _dp, _dp]
    lib.oracle_block_potential.argtypes = [d, d, i64, _dp, _dp, _dp, _dp, i32, i32, _dp, _dp]
    lib.oracle_bin_density.argtypes = [d, d, i64, _dp, _dp, _dp, _dp, i32, _dp]
    lib.oracle_bin_coeffs.argtypes = [d, d, i32, _dp, i32, i32, _dp]
    lib.oracle_bin_field.argtypes = [d, d, i32, i32, i32, _dp, _dp, _dp, _dp]
    lib.oracle_bin_density_at.argtypes = [d, d, i64, _dp, _dp, _dp, _dp, i32, i64, _ip, _ip, _dp]
    lib.oracle_bin_coeffs_at.argtypes = [d, d, i32, _dp, i64, _ip, _ip, _dp]
    lib.oracle_bin_interp.argtypes = [d, d, i64, _dp, _dp, _dp, _dp, i32, _dp, _dp, _dp, _dp, _dp, _dp]
    lib.oracle_num_threads.argtypes = []
    lib.oracle_set_num_threads.argtypes = [ctypes.c_int]
    lib.oracle_set_num_threads.restype = None
    for f in ("oracle_coeffs", "oracle_energy", "oracle_grad", "oracle_grad_sampled",
              "oracle_coeffs_sampled", "oracle_coeffs_sampled_full", "oracle_raw_moments",
              "oracle_coef_factors", "oracle_point_field", "oracle_block_potential", "oracle_bin_field",
              "oracle_num_threads"):
        getattr(lib, f).restype = ctypes.c_int
    _lib = lib
    return lib


def _f64(a):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    return a, a.ctypes.data_as(_dp)


def _check(st, what):
    if st != 0:
        raise RuntimeError(f"oracle {what} failed with status {st}")


def num_threads() -> int:
    return int(_load().oracle_num_threads())


def set_num_threads(k: int) -> None:
    """Threads of the oracle's later parallel loops (OpenMP); k <= 0 leaves the setting unchanged."""
    _load().oracle_set_num_threads(int(k))


def coeffs(W, H, x, y, w, h, Mu, Mp):
    """Return (a, I): coefficients a_up and density moments I_up, both [Mu, Mp]."""
    lib = _load()
    xs = [_f64(v) for v in (x, y, w, h)]
    n = xs[0][0].shape[0]
    a = np.zeros((Mu, Mp))
    I = np.zeros((Mu, Mp))
    _check(lib.oracle_coeffs(W, H, n, *[p for _, p in xs], Mu, Mp, a.ctypes.data_as(_dp),
                             I.ctypes.data_as(_dp)), "coeffs")
    return a, I


def energy(W, H, x, y, w, h, Mu, Mp):
    """Return (E, a, I)."""
    lib = _load()
    xs = [_f64(v) for v in (x, y, w, h)]
    n = xs[0][0].shape[0]
    a = np.zeros((Mu, Mp))
    I = np.zeros((Mu, Mp))
    E = ctypes.c_double(0.0)
    _check(lib.oracle_energy(W, H, n, *[p for _, p in xs], Mu, Mp, ctypes.byref(E),
                             a.ctypes.data_as(_dp), I.ctypes.data_as(_dp)), "energy")
    return float(E.value), a, I


def grad(W, H, x, y, w, h, a):
    """dE/dx_i, dE/dy_i for all blocks, given the oracle's coefficients a [Mu, Mp]."""
    lib = _load()
    xs = [_f64(v) for v in (x, y, w, h)]
    n = xs[0][0].shape[0]
    a, pa = _f64(a)
    gx = np.zeros(n)
    gy = np.zeros(n)
    _check(lib.oracle_grad(W, H, n, *[p for _, p in xs], a.shape[0], a.shape[1], pa,
                           gx.ctypes.data_as(_dp), gy.ctypes.data_as(_dp)), "grad")
    return gx, gy


def grad_sampled(W, H, x, y, w, h, a, idx):
    lib = _load()
    xs = [_f64(v) for v in (x, y, w, h)]
    a, pa = _f64(a)
    idx = np.ascontiguousarray(np.asarray(idx, dtype=np.int64))
    gx = np.zeros(idx.shape[0])
    gy = np.zeros(idx.shape[0])
    _check(lib.oracle_grad_sampled(W, H, *[p for _, p in xs], a.shape[0], a.shape[1], pa, idx.shape[0],
                                   idx.ctypes.data_as(_lp), gx.ctypes.data_as(_dp),
                                   gy.ctypes.data_as(_dp)), "grad_sampled")
    return gx, gy


def coeffs_sampled(W, H, x, y, w, h, us, ps):
    """Coefficients a_{us[k], ps[k]} and moments, each by an O(n) direct sum."""
    lib = _load()
    xs = [_f64(v) for v in (x, y, w, h)]
    n = xs[0][0].shape[0]
    us = np.ascontiguousarray(np.asarray(us, dtype=np.int32))
    ps = np.ascontiguousarray(np.asarray(ps, dtype=np.int32))
    a = np.zeros(us.shape[0])
    I = np.zeros(us.shape[0])
    _check(lib.oracle_coeffs_sampled(W, H, n, *[p for _, p in xs], us.shape[0], us.ctypes.data_as(_ip),
                                     ps.ctypes.data_as(_ip), a.ctypes.data_as(_dp),
                                     I.ctypes.data_as(_dp)), "coeffs_sampled")
    return a, I


def raw_moments(W, H, x, y, w, h, Mu, Mp):
    """Raw block sums R[u, p] = sum_i S'_iu T'_ip (S'_i0 = w_i, T'_i0 = h_i): the moments with
    their frequency factors taken out, of the same magnitude over the whole (u, p) plane."""
    lib = _load()
    xs = [_f64(v) for v in (x, y, w, h)]
    n = xs[0][0].shape[0]
    R = np.zeros((Mu, Mp))
    _check(lib.oracle_raw_moments(W, H, n, *[p for _, p in xs], Mu, Mp, R.ctypes.data_as(_dp)), "raw_moments")
    return R


def coef_factors(W, H, Mu, Mp):
    """Prefactors f[u, p] of the closed-form coefficients, a_up = f_up R_up (f_00 = 0)."""
    f = np.zeros((Mu, Mp))
    _check(_load().oracle_coef_factors(W, H, Mu, Mp, f.ctypes.data_as(_dp)), "coef_factors")
    return f


def coeffs_sampled_full(W, H, x, y, w, h, us, ps):
    """(a, R, Rabs) at the sampled (us[k], ps[k]): the coefficient, the raw sum R = sum_i S'_iu T'_ip
    and its absolute counterpart Rabs = sum_i |S'_iu T'_ip| (the scale of the sum's rounding errors)."""
    lib = _load()
    xs = [_f64(v) for v in (x, y, w, h)]
    n = xs[0][0].shape[0]
    us = np.ascontiguousarray(np.asarray(us, dtype=np.int32))
    ps = np.ascontiguousarray(np.asarray(ps, dtype=np.int32))
    k = us.shape[0]
    a, R, Ra = np.zeros(k), np.zeros(k), np.zeros(k)
    _check(lib.oracle_coeffs_sampled_full(W, H, n, *[p for _, p in xs], k, us.ctypes.data_as(_ip),
                                          ps.ctypes.data_as(_ip), a.ctypes.data_as(_dp), None,
                                          R.ctypes.data_as(_dp), Ra.ctypes.data_as(_dp)), "coeffs_sampled_full")
    return a, R, Ra


def point_field(W, H, a, px, py):
    """psi, xi_x, xi_y at the points (px[k], py[k])."""
    lib = _load()
    a, pa = _f64(a)
    px, ppx = _f64(px)
    py, ppy = _f64(py)
    n = px.shape[0]
    psi, ex, ey = np.zeros(n), np.zeros(n), np.zeros(n)
    _check(lib.oracle_point_field(W, H, a.shape[0], a.shape[1], pa, n, ppx, ppy, psi.ctypes.data_as(_dp),
                                  ex.ctypes.data_as(_dp), ey.ctypes.data_as(_dp)), "point_field")
    return psi, ex, ey


def block_potential(W, H, x, y, w, h, a):
    """N_i = integral of psi over block i."""
    lib = _load()
    xs = [_f64(v) for v in (x, y, w, h)]
    n = xs[0][0].shape[0]
    a, pa = _f64(a)
    N = np.zeros(n)
    _check(lib.oracle_block_potential(W, H, n, *[p for _, p in xs], a.shape[0], a.shape[1], pa,
                                      N.ctypes.data_as(_dp)), "block_potential")
    return N


def bin_density(W, H, x, y, w, h, m):
    """Bin densities P[l, j] of an m x m grid (Sec. III-D): exact overlap areas over the bin area."""
    lib = _load()
    xs = [_f64(v) for v in (x, y, w, h)]
    n = xs[0][0].shape[0]
    P = np.zeros((m, m))
    _check(lib.oracle_bin_density(W, H, n, *[p for _, p in xs], m, P.ctypes.data_as(_dp)), "bin_density")
    return P


def bin_coeffs(W, H, P, Mu, Mp):
    """Binned coefficients a[u, p] (Sec. III-D, eqs. disa-a..d) of the bin densities P (m x m)."""
    lib = _load()
    P, pP = _f64(P)
    m = P.shape[0]
    a = np.zeros((Mu, Mp))
    _check(lib.oracle_bin_coeffs(W, H, m, pP, Mu, Mp, a.ctypes.data_as(_dp)), "bin_coeffs")
    return a


def bin_field(W, H, m, a):
    """psi, xi_x, xi_y at the centres of the m x m bins (eqs. dis-psi1, dis-ksi), truncated at a."""
    lib = _load()
    a, pa = _f64(a)
    Mu, Mp = a.shape
    psi, xix, xiy = np.zeros((m, m)), np.zeros((m, m)), np.zeros((m, m))
    _check(lib.oracle_bin_field(W, H, m, Mu, Mp, pa, psi.ctypes.data_as(_dp), xix.ctypes.data_as(_dp),
                                xiy.ctypes.data_as(_dp)), "bin_field")
    return psi, xix, xiy


def bin_density_at(W, H, x, y, w, h, m, ls, js):
    """Selected bin densities P[ls[k], js[k]] (for grids too large for bin_density)."""
    lib = _load()
    xs = [_f64(v) for v in (x, y, w, h)]
    n = xs[0][0].shape[0]
    ls = np.ascontiguousarray(ls, dtype=np.int32)
    js = np.ascontiguousarray(js, dtype=np.int32)
    out = np.zeros(len(ls))
    _check(lib.oracle_bin_density_at(W, H, n, *[p for _, p in xs], m, len(ls), ls.ctypes.data_as(_ip),
                                     js.ctypes.data_as(_ip), out.ctypes.data_as(_dp)), "bin_density_at")
    return out


def bin_coeffs_at(W, H, P, us, ps):
    """Selected binned coefficients a[us[k], ps[k]] of the bin densities P (m x m)."""
    lib = _load()
    P, pP = _f64(P)
    us = np.ascontiguousarray(us, dtype=np.int32)
    ps = np.ascontiguousarray(ps, dtype=np.int32)
    out = np.zeros(len(us))
    _check(lib.oracle_bin_coeffs_at(W, H, P.shape[0], pP, len(us), us.ctypes.data_as(_ip), ps.ctypes.data_as(_ip),
                                    out.ctypes.data_as(_dp)), "bin_coeffs_at")
    return out


def bin_interp(W, H, x, y, w, h, m, psi=None, xix=None, xiy=None):
    """Block values from bin values: (N, gx, gy), N_i = sum over the bins of |block i cap bin| psi,
    gx_i = -sum |block i cap bin| xi_x, gy_i likewise; an output is None when its field is None."""
    lib = _load()
    xs = [_f64(v) for v in (x, y, w, h)]
    n = xs[0][0].shape[0]
    ins, outs = [], []
    for f in (psi, xix, xiy):
        if f is None:
            ins.append(None)
            outs.append(None)
        else:
            f, _ = _f64(f)
            if f.shape != (m, m):
                raise ValueError("bin fields must be m x m")
            ins.append(f)
            outs.append(np.zeros(n))
    ptr = lambda a: None if a is None else a.ctypes.data_as(_dp)
    _check(lib.oracle_bin_interp(W, H, n, *[p for _, p in xs], m, *[ptr(a) for a in ins], *[ptr(a) for a in outs]),
           "bin_interp")
    return tuple(outs)
