"""Python binding of libpplace (include/pplace.h): argument marshalling only.

Every step of the computation runs in the HIP kernels of ``libpplace.so``; this module passes
device pointers of contiguous FP64 torch tensors, a caller-sized workspace and torch's current
HIP stream.  PyTorch supplies memory and streams, nothing else.  If the library has not been
built, every entry point raises instead of computing anything another way.

The method (arXiv 2307.12041, Sec. III-A): on the region [0, W] x [0, H] with n rectangular blocks,
the potential is psi = sum_{u<Mu, p<Mp} a_up cos(u pi x / W) cos(p pi y / H) with the closed-form
coefficients of the exact block density; the energy is E = 1/2 iint rho psi and the gradient of E
with respect to the block centres is minus the field (eq. ksi) integrated over each block.
"""
from __future__ import annotations

import ctypes
import os

import torch

__all__ = ["PRECISIONS", "BASIS_MODES", "PPError", "library_path", "load", "workspace_size", "coeffs",
           "energy", "energy_static", "field", "point_field", "block_potential", "PPEnergy", "energy_autograd", "timing_enable",
           "timing_query", "mfma_calibrate", "bin_workspace_size", "bin_density", "bin_coeffs", "bin_field"]

_HERE = os.path.dirname(os.path.abspath(__file__))
# PP_LIBRARY names another build of the same library (the host-sanitizer test uses it).
_LIB_PATH = os.environ.get("PP_LIBRARY") or os.path.join(_HERE, "libpplace.so")

PRECISIONS = {"fp64": 0, "fp32": 1, "bf16": 2, "bf16x3": 3, "fp8": 4, "fp8x3": 5, "bf16mix": 6}
BASIS_MODES = {"recompute": 0, "store": 1}

PP_OK = 0
EXPORTS = ("pp_workspace_size", "pp_coeffs", "pp_energy", "pp_energy_static", "pp_field", "pp_point_field",
           "pp_block_potential",
           "pp_strerror", "pp_timing_enable", "pp_timing_query", "pp_mfma_calibrate", "pp_bin_workspace_size",
           "pp_bin_density",
           "pp_bin_coeffs", "pp_bin_field", "pp_bin_interp")


class PPError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__(f"{what}: {_strerror(status)} (status {status})")


class PPProblem(ctypes.Structure):
    _fields_ = [("W", ctypes.c_double), ("H", ctypes.c_double), ("n", ctypes.c_int64),
                ("Mu", ctypes.c_int32), ("Mp", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("basis_mode", ctypes.c_int32)]


class PPBinProblem(ctypes.Structure):
    _fields_ = [("W", ctypes.c_double), ("H", ctypes.c_double), ("n", ctypes.c_int64), ("m", ctypes.c_int32),
                ("Mu", ctypes.c_int32), ("Mp", ctypes.c_int32)]


_lib = None


def library_path() -> str:
    return _LIB_PATH


def load():
    """Load libpplace.so and declare the C signatures.  Raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise RuntimeError(f"{_LIB_PATH} is not built; run `python -c 'import __graft_entry__ as g; g.build()'`")
    lib = ctypes.CDLL(_LIB_PATH)
    P = ctypes.POINTER(PPProblem)
    vp, sz = ctypes.c_void_p, ctypes.c_size_t
    lib.pp_workspace_size.argtypes = [P, ctypes.POINTER(sz)]
    lib.pp_coeffs.argtypes = [P, vp, vp, vp, vp, vp, vp, sz, vp]
    lib.pp_energy.argtypes = [P, vp, vp, vp, vp, vp, vp, vp, sz, vp]
    lib.pp_energy_static.argtypes = [P, vp, vp, vp, vp, vp, vp, vp]
    lib.pp_field.argtypes = [P, vp, vp, vp, vp, vp, vp, vp, vp, vp, sz, vp]
    lib.pp_point_field.argtypes = [P, vp, vp, vp, vp, vp, vp, vp, sz, vp]
    lib.pp_block_potential.argtypes = [P, vp, vp, vp, vp, vp, vp, vp, sz, vp]
    lib.pp_strerror.argtypes = [ctypes.c_int]
    lib.pp_strerror.restype = ctypes.c_char_p
    lib.pp_timing_enable.argtypes = [ctypes.c_int]
    lib.pp_timing_enable.restype = ctypes.c_int
    lib.pp_timing_query.argtypes = [ctypes.c_char_p, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int)]
    lib.pp_timing_query.restype = ctypes.c_int
    lib.pp_mfma_calibrate.argtypes = [ctypes.c_int, ctypes.c_int, vp, vp]
    lib.pp_mfma_calibrate.restype = ctypes.c_int
    B = ctypes.POINTER(PPBinProblem)
    lib.pp_bin_workspace_size.argtypes = [B, ctypes.POINTER(sz)]
    lib.pp_bin_density.argtypes = [B, vp, vp, vp, vp, vp, vp, sz, vp]
    lib.pp_bin_coeffs.argtypes = [B, vp, vp, vp, sz, vp]
    lib.pp_bin_field.argtypes = [B, vp, vp, vp, vp, vp, sz, vp]
    lib.pp_bin_interp.argtypes = [B, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, sz, vp]
    for f in ("pp_workspace_size", "pp_coeffs", "pp_energy", "pp_energy_static", "pp_field", "pp_point_field",
              "pp_block_potential",
              "pp_bin_workspace_size", "pp_bin_density", "pp_bin_coeffs", "pp_bin_field", "pp_bin_interp"):
        getattr(lib, f).restype = ctypes.c_int
    _lib = lib
    return lib


def _strerror(status: int) -> str:
    try:
        return load().pp_strerror(int(status)).decode()
    except Exception:  # pragma: no cover
        return "unknown"


def _problem(W, H, n, Mu, Mp, precision, basis) -> PPProblem:
    if precision not in PRECISIONS:
        raise ValueError(f"unknown precision {precision!r}; one of {sorted(PRECISIONS)}")
    if basis not in BASIS_MODES:
        raise ValueError(f"unknown basis mode {basis!r}; one of {sorted(BASIS_MODES)}")
    return PPProblem(float(W), float(H), int(n), int(Mu), int(Mp), PRECISIONS[precision], BASIS_MODES[basis])


def workspace_size(W, H, n, Mu, Mp, precision="fp64", basis="recompute") -> int:
    P = _problem(W, H, n, Mu, Mp, precision, basis)
    out = ctypes.c_size_t(0)
    st = load().pp_workspace_size(ctypes.byref(P), ctypes.byref(out))
    if st != PP_OK:
        raise PPError(st, "pp_workspace_size")
    return int(out.value)


def _blocks(x, y, w, h):
    ts = (x, y, w, h)
    dev = x.device
    n = x.shape[0]
    for t in ts:
        if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or t.dim() != 1:
            raise TypeError("x, y, w, h must be 1-D float64 tensors")
        if t.device != dev or t.shape[0] != n or not t.is_contiguous():
            raise ValueError("x, y, w, h must be contiguous, on one device, of equal length")
    if dev.type != "cuda":
        raise ValueError("x, y, w, h must live on a GPU (HIP) device")
    return dev, n


def _vp(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream(dev):
    return ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)


def _workspace(P, dev, workspace=None):
    """The caller's workspace if given (a uint8 device tensor, large enough), else a fresh one."""
    nbytes = ctypes.c_size_t(0)
    st = load().pp_workspace_size(ctypes.byref(P), ctypes.byref(nbytes))
    if st != PP_OK:
        raise PPError(st, "pp_workspace_size")
    if workspace is not None:
        if workspace.device != dev or workspace.dtype != torch.uint8 or not workspace.is_contiguous():
            raise ValueError("workspace must be a contiguous uint8 tensor on the blocks' device")
        return workspace, int(workspace.numel())
    ws = torch.empty(max(int(nbytes.value), 1), dtype=torch.uint8, device=dev)
    return ws, int(nbytes.value)


def coeffs(x, y, w, h, *, W, H, Mu, Mp, precision="fp64", basis="recompute", workspace=None):
    """Series coefficients a [Mu, Mp] (FP64, on the device of x)."""
    dev, n = _blocks(x, y, w, h)
    P = _problem(W, H, n, Mu, Mp, precision, basis)
    a = torch.empty((Mu, Mp), dtype=torch.float64, device=dev)
    ws, nb = _workspace(P, dev, workspace)
    with torch.cuda.device(dev):
        st = load().pp_coeffs(ctypes.byref(P), _vp(x), _vp(y), _vp(w), _vp(h), _vp(a), _vp(ws), nb, _stream(dev))
    if st != PP_OK:
        raise PPError(st, "pp_coeffs")
    return a


def energy(x, y, w, h, *, W, H, Mu, Mp, precision="fp64", basis="recompute", want_coeffs=True, workspace=None):
    """Energy E (0-d FP64 tensor) and, if asked, the coefficients a [Mu, Mp]."""
    dev, n = _blocks(x, y, w, h)
    P = _problem(W, H, n, Mu, Mp, precision, basis)
    E = torch.empty((), dtype=torch.float64, device=dev)
    a = torch.empty((Mu, Mp), dtype=torch.float64, device=dev) if want_coeffs else None
    ws, nb = _workspace(P, dev, workspace)
    with torch.cuda.device(dev):
        st = load().pp_energy(ctypes.byref(P), _vp(x), _vp(y), _vp(w), _vp(h), _vp(E), _vp(a), _vp(ws), nb,
                              _stream(dev))
    if st != PP_OK:
        raise PPError(st, "pp_energy")
    return E, a


def energy_static(x, y, w, h, *, W, H, Mu, Mp, precision="fp64", want_coeffs=True):
    """energy() through pp_energy_static: the library's own per-device static scratch serves as the
    workspace (no allocation inside the call; at most PP_STATIC_SCRATCH_BYTES)."""
    dev, n = _blocks(x, y, w, h)
    P = _problem(W, H, n, Mu, Mp, precision, "recompute")
    E = torch.empty((), dtype=torch.float64, device=dev)
    a = torch.empty((Mu, Mp), dtype=torch.float64, device=dev) if want_coeffs else None
    with torch.cuda.device(dev):
        st = load().pp_energy_static(ctypes.byref(P), _vp(x), _vp(y), _vp(w), _vp(h), _vp(E), _vp(a), _stream(dev))
    if st != PP_OK:
        raise PPError(st, "pp_energy_static")
    return E, a


def field(x, y, w, h, a, *, W, H, precision="fp64", basis="recompute", dE=None, workspace=None):
    """Per-block gradient (gx, gy) = dE * (dE/dx_i, dE/dy_i); the force on block i is -(gx, gy).

    With basis "store", `workspace` must be the one that the energy (or coeffs) call of the same
    blocks filled: the gradient reads the basis tables that call left in it."""
    if basis == "store" and workspace is None:
        raise ValueError("basis='store': pass the workspace that energy()/coeffs() of the same blocks filled")
    dev, n = _blocks(x, y, w, h)
    if a.dtype != torch.float64 or a.dim() != 2 or not a.is_contiguous() or a.device != dev:
        raise ValueError("a must be a contiguous [Mu, Mp] float64 tensor on the blocks' device")
    Mu, Mp = a.shape
    P = _problem(W, H, n, Mu, Mp, precision, basis)
    if dE is not None:
        dE = dE.to(device=dev, dtype=torch.float64).contiguous()
    gx = torch.empty(n, dtype=torch.float64, device=dev)
    gy = torch.empty(n, dtype=torch.float64, device=dev)
    ws, nb = _workspace(P, dev, workspace)
    with torch.cuda.device(dev):
        st = load().pp_field(ctypes.byref(P), _vp(x), _vp(y), _vp(w), _vp(h), _vp(a), _vp(dE), _vp(gx), _vp(gy),
                             _vp(ws), nb, _stream(dev))
    if st != PP_OK:
        raise PPError(st, "pp_field")
    return gx, gy


def _coeff_arg(a, dev):
    if not isinstance(a, torch.Tensor) or a.dtype != torch.float64 or a.dim() != 2 or not a.is_contiguous() \
            or a.device != dev:
        raise ValueError("a must be a contiguous [Mu, Mp] float64 tensor on the points' device")
    return a.shape


def point_field(px, py, a, *, W, H, precision="fp64", want=("psi", "xix", "xiy"), workspace=None):
    """Point values (psi, xix, xiy) of the potential and the field xi = -grad psi at (px[k], py[k]);
    an output not named in `want` is None."""
    for t in (px, py):
        if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or t.dim() != 1 or not t.is_contiguous():
            raise TypeError("px, py must be contiguous 1-D float64 tensors")
    dev, n = px.device, px.shape[0]
    if py.device != dev or py.shape[0] != n or dev.type != "cuda":
        raise ValueError("px, py must be of equal length on one GPU (HIP) device")
    Mu, Mp = _coeff_arg(a, dev)
    P = _problem(W, H, n, Mu, Mp, precision, "recompute")
    outs = {k: (torch.empty(n, dtype=torch.float64, device=dev) if k in want else None)
            for k in ("psi", "xix", "xiy")}
    ws, nb = _workspace(P, dev, workspace)
    with torch.cuda.device(dev):
        st = load().pp_point_field(ctypes.byref(P), _vp(px), _vp(py), _vp(a), _vp(outs["psi"]), _vp(outs["xix"]),
                                   _vp(outs["xiy"]), _vp(ws), nb, _stream(dev))
    if st != PP_OK:
        raise PPError(st, "pp_point_field")
    return outs["psi"], outs["xix"], outs["xiy"]


def block_potential(x, y, w, h, a, *, W, H, precision="fp64", workspace=None):
    """Per-block potential energies N_i = integral of psi over block i (E = 1/2 sum_i N_i)."""
    dev, n = _blocks(x, y, w, h)
    Mu, Mp = _coeff_arg(a, dev)
    P = _problem(W, H, n, Mu, Mp, precision, "recompute")
    N = torch.empty(n, dtype=torch.float64, device=dev)
    ws, nb = _workspace(P, dev, workspace)
    with torch.cuda.device(dev):
        st = load().pp_block_potential(ctypes.byref(P), _vp(x), _vp(y), _vp(w), _vp(h), _vp(a), _vp(N), _vp(ws),
                                       nb, _stream(dev))
    if st != PP_OK:
        raise PPError(st, "pp_block_potential")
    return N


# ------------------------------------------------------------------------------------------------
# Bin scheme (Sec. III-D), the comparison path: m x m bins, FP64 throughout.
# ------------------------------------------------------------------------------------------------
def _bin_problem(W, H, n, m, Mu, Mp) -> PPBinProblem:
    return PPBinProblem(float(W), float(H), int(n), int(m), int(Mu), int(Mp))


def bin_workspace_size(W, H, n, m, Mu=None, Mp=None) -> int:
    B = _bin_problem(W, H, n, m, m if Mu is None else Mu, m if Mp is None else Mp)
    out = ctypes.c_size_t(0)
    st = load().pp_bin_workspace_size(ctypes.byref(B), ctypes.byref(out))
    if st != PP_OK:
        raise PPError(st, "pp_bin_workspace_size")
    return int(out.value)


def _bin_ws(B, dev, workspace):
    nbytes = ctypes.c_size_t(0)
    st = load().pp_bin_workspace_size(ctypes.byref(B), ctypes.byref(nbytes))
    if st != PP_OK:
        raise PPError(st, "pp_bin_workspace_size")
    if workspace is not None:
        if workspace.device != dev or workspace.dtype != torch.uint8 or not workspace.is_contiguous():
            raise ValueError("workspace must be a contiguous uint8 tensor on the data's device")
        return workspace, int(workspace.numel())
    return torch.empty(max(int(nbytes.value), 1), dtype=torch.uint8, device=dev), int(nbytes.value)


def _bin_matrix(t, rows, cols, dev, name):
    if (not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or tuple(t.shape) != (rows, cols)
            or not t.is_contiguous() or t.device != dev):
        raise ValueError(f"{name} must be a contiguous float64 [{rows}, {cols}] tensor on the GPU")


def bin_density(x, y, w, h, *, W, H, m, workspace=None):
    """Bin densities P[l, j] of an m x m grid: exact overlap areas of the blocks over the bin area."""
    dev, n = _blocks(x, y, w, h)
    B = _bin_problem(W, H, n, m, 1, 1)
    P = torch.empty((m, m), dtype=torch.float64, device=dev)
    ws, nb = _bin_ws(B, dev, workspace)
    with torch.cuda.device(dev):
        st = load().pp_bin_density(ctypes.byref(B), _vp(x), _vp(y), _vp(w), _vp(h), _vp(P), _vp(ws), nb,
                                   _stream(dev))
    if st != PP_OK:
        raise PPError(st, "pp_bin_density")
    return P


def bin_coeffs(P, *, W, H, Mu, Mp, workspace=None):
    """Binned coefficients a[u, p], u < Mu, p < Mp (eqs. disa-a..d) of the m x m bin densities P."""
    if not isinstance(P, torch.Tensor) or P.dim() != 2:
        raise ValueError("P must be a 2-D tensor")
    m, dev = P.shape[0], P.device
    _bin_matrix(P, m, m, dev, "P")
    B = _bin_problem(W, H, 0, m, Mu, Mp)
    a = torch.empty((Mu, Mp), dtype=torch.float64, device=dev)
    ws, nb = _bin_ws(B, dev, workspace)
    with torch.cuda.device(dev):
        st = load().pp_bin_coeffs(ctypes.byref(B), _vp(P), _vp(a), _vp(ws), nb, _stream(dev))
    if st != PP_OK:
        raise PPError(st, "pp_bin_coeffs")
    return a


def bin_field(a, *, W, H, m, want=("psi", "xix", "xiy"), workspace=None):
    """psi, xi_x, xi_y at the centres of the m x m bins (eqs. dis-psi1, dis-ksi); outputs not named in
    `want` are None."""
    if not isinstance(a, torch.Tensor) or a.dim() != 2:
        raise ValueError("a must be a 2-D tensor")
    Mu, Mp = a.shape
    dev = a.device
    _bin_matrix(a, Mu, Mp, dev, "a")
    B = _bin_problem(W, H, 0, m, Mu, Mp)
    outs = {k: (torch.empty((m, m), dtype=torch.float64, device=dev) if k in want else None)
            for k in ("psi", "xix", "xiy")}
    ws, nb = _bin_ws(B, dev, workspace)
    with torch.cuda.device(dev):
        st = load().pp_bin_field(ctypes.byref(B), _vp(a), _vp(outs["psi"]), _vp(outs["xix"]), _vp(outs["xiy"]),
                                 _vp(ws), nb, _stream(dev))
    if st != PP_OK:
        raise PPError(st, "pp_bin_field")
    return outs["psi"], outs["xix"], outs["xiy"]


def bin_interp(x, y, w, h, psi=None, xix=None, xiy=None, *, W, H, workspace=None):
    """Block values from bin values (N, gx, gy): N_i = sum over the bins of |block i cap bin| psi,
    gx_i = -sum |block i cap bin| xi_x, gy_i likewise; an output is None when its field is None."""
    dev, n = _blocks(x, y, w, h)
    fields = (psi, xix, xiy)
    given = [f for f in fields if f is not None]
    if not given:
        raise ValueError("give at least one of psi, xix, xiy")
    m = given[0].shape[0]
    for f, name in zip(fields, ("psi", "xix", "xiy")):
        if f is not None:
            _bin_matrix(f, m, m, dev, name)
    B = _bin_problem(W, H, n, m, 1, 1)
    outs = [torch.empty(n, dtype=torch.float64, device=dev) if f is not None else None for f in fields]
    ws, nb = _bin_ws(B, dev, workspace)
    with torch.cuda.device(dev):
        st = load().pp_bin_interp(ctypes.byref(B), _vp(x), _vp(y), _vp(w), _vp(h), *[_vp(f) for f in fields],
                                  *[_vp(o) for o in outs], _vp(ws), nb, _stream(dev))
    if st != PP_OK:
        raise PPError(st, "pp_bin_interp")
    return tuple(outs)


def timing_enable(on: bool) -> None:
    """Start (or stop) HIP-event timing of every kernel launch of the library; clears records."""
    load().pp_timing_enable(1 if on else 0)


def timing_query(stage: str):
    """(total_ms, launches) recorded for one stage since timing_enable (waits for the events)."""
    ms = ctypes.c_double(0.0)
    cnt = ctypes.c_int(0)
    st = load().pp_timing_query(stage.encode(), ctypes.byref(ms), ctypes.byref(cnt))
    if st != PP_OK:
        raise PPError(st, "pp_timing_query")
    return float(ms.value), int(cnt.value)


def mfma_calibrate(out, *, workgroups, iters):
    """Enqueue the matrix-core calibration kernel on torch's current stream of out's device (out: a
    contiguous float32 CUDA tensor of at least workgroups * 256 elements); time it with events on that
    stream.  The launch executes workgroups * 4 * 16 * iters * 32768 bf16 flops."""
    if not (isinstance(out, torch.Tensor) and out.is_cuda and out.dtype == torch.float32 and out.is_contiguous()):
        raise TypeError("out must be a contiguous float32 CUDA tensor")
    if out.numel() < workgroups * 256:
        raise ValueError("out holds fewer than workgroups * 256 floats")
    with torch.cuda.device(out.device):
        st = load().pp_mfma_calibrate(int(workgroups), int(iters), _vp(out), _stream(out.device))
    if st != PP_OK:
        raise PPError(st, "pp_mfma_calibrate")


class PPEnergy(torch.autograd.Function):
    """E(x, y) with a backward that maps dE to per-block gradients through pp_field.

    With basis "recompute" the forward keeps only the coefficients a (Mu*Mp FP64) and the backward
    regenerates every basis tile on chip.  With basis "store" the forward's workspace, which holds
    the n x M basis tables, is kept until the backward reads them.  w and h are not differentiated."""

    @staticmethod
    def forward(ctx, x, y, w, h, W, H, Mu, Mp, precision, basis):
        ws = None
        if basis == "store":
            ws = torch.empty(max(workspace_size(W, H, x.shape[0], Mu, Mp, precision, basis), 1), dtype=torch.uint8,
                             device=x.device)
        E, a = energy(x, y, w, h, W=W, H=H, Mu=Mu, Mp=Mp, precision=precision, basis=basis, workspace=ws)
        ctx.save_for_backward(x, y, w, h, a)
        ctx.cfg = (W, H, precision, basis)
        ctx.ws = ws
        return E

    @staticmethod
    def backward(ctx, gE):
        x, y, w, h, a = ctx.saved_tensors
        W, H, precision, basis = ctx.cfg
        gx, gy = field(x.detach(), y.detach(), w.detach(), h.detach(), a, W=W, H=H, precision=precision,
                       basis=basis, dE=gE.detach(), workspace=ctx.ws)
        ctx.ws = None
        return gx, gy, None, None, None, None, None, None, None, None


def energy_autograd(x, y, w, h, *, W, H, Mu, Mp, precision="fp64", basis="recompute"):
    """Differentiable energy: ``E.backward()`` fills x.grad, y.grad with dE/dx_i, dE/dy_i."""
    return PPEnergy.apply(x, y, w, h, W, H, Mu, Mp, precision, basis)
