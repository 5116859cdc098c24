// A plain C++ caller of the C ABI of include/pplace.h, as an application without Python or torch
// would use it: device memory and a stream from the HIP runtime, the workspace sized by
// pp_workspace_size, then pp_energy and pp_field on that stream, and the results copied back.
// Built as a small shared library so that a test can drive it in-process.
#include <hip/hip_runtime.h>
#include <stdio.h>
#include <string.h>

#include "pplace.h"

namespace {

struct Dev {
    void *p = nullptr;
    ~Dev() {
        if (p) (void)hipFree(p);
    }
};

int hip_fail(hipError_t e, const char *what, char *msg, int len) {
    snprintf(msg, (size_t)len, "%s: %s", what, hipGetErrorString(e));
    return -100;
}

}  // namespace

// Energy and gradient of n blocks given in host memory.  Returns 0, a pp status (< 0, message from
// pp_strerror) or -100 for a HIP runtime failure (message names the call).  E: one double; a: Mu*Mp;
// gx, gy: n doubles; all host memory owned by the caller.
extern "C" int abi_caller_run(double W, double H, int64_t n, int Mu, int Mp, int precision, const double *x,
                              const double *y, const double *w, const double *h, double *E, double *a, double *gx,
                              double *gy, char *msg, int msg_len) {
    msg[0] = 0;
    pp_problem P;
    P.W = W;
    P.H = H;
    P.n = n;
    P.Mu = Mu;
    P.Mp = Mp;
    P.precision = precision;
    P.basis_mode = PP_BASIS_RECOMPUTE;
    size_t ws_bytes = 0;
    int st = pp_workspace_size(&P, &ws_bytes);
    if (st != PP_OK) {
        snprintf(msg, (size_t)msg_len, "pp_workspace_size: %s", pp_strerror(st));
        return st;
    }
    const size_t nb = (size_t)n * sizeof(double), mb = (size_t)Mu * (size_t)Mp * sizeof(double);
    Dev dx, dy, dw, dh, dE, da, dgx, dgy, dws;
    hipError_t e;
    Dev *in[4] = {&dx, &dy, &dw, &dh};
    const double *src[4] = {x, y, w, h};
    for (int k = 0; k < 4; ++k) {
        if ((e = hipMalloc(&in[k]->p, nb > 0 ? nb : 8)) != hipSuccess) return hip_fail(e, "hipMalloc", msg, msg_len);
        if (nb > 0 && (e = hipMemcpy(in[k]->p, src[k], nb, hipMemcpyHostToDevice)) != hipSuccess)
            return hip_fail(e, "hipMemcpy", msg, msg_len);
    }
    if ((e = hipMalloc(&dE.p, sizeof(double))) != hipSuccess || (e = hipMalloc(&da.p, mb)) != hipSuccess ||
        (e = hipMalloc(&dgx.p, nb > 0 ? nb : 8)) != hipSuccess || (e = hipMalloc(&dgy.p, nb > 0 ? nb : 8)) != hipSuccess ||
        (e = hipMalloc(&dws.p, ws_bytes > 0 ? ws_bytes : 256)) != hipSuccess)
        return hip_fail(e, "hipMalloc", msg, msg_len);
    hipStream_t s;
    if ((e = hipStreamCreate(&s)) != hipSuccess) return hip_fail(e, "hipStreamCreate", msg, msg_len);
    st = pp_energy(&P, (const double *)dx.p, (const double *)dy.p, (const double *)dw.p, (const double *)dh.p,
                   (double *)dE.p, (double *)da.p, dws.p, ws_bytes, s);
    if (st == PP_OK)
        st = pp_field(&P, (const double *)dx.p, (const double *)dy.p, (const double *)dw.p, (const double *)dh.p,
                      (const double *)da.p, nullptr, (double *)dgx.p, (double *)dgy.p, dws.p, ws_bytes, s);
    e = hipStreamSynchronize(s);
    (void)hipStreamDestroy(s);
    if (st != PP_OK) {
        snprintf(msg, (size_t)msg_len, "pp call: %s", pp_strerror(st));
        return st;
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize", msg, msg_len);
    if ((e = hipMemcpy(E, dE.p, sizeof(double), hipMemcpyDeviceToHost)) != hipSuccess ||
        (e = hipMemcpy(a, da.p, mb, hipMemcpyDeviceToHost)) != hipSuccess ||
        (nb > 0 && (e = hipMemcpy(gx, dgx.p, nb, hipMemcpyDeviceToHost)) != hipSuccess) ||
        (nb > 0 && (e = hipMemcpy(gy, dgy.p, nb, hipMemcpyDeviceToHost)) != hipSuccess))
        return hip_fail(e, "hipMemcpy", msg, msg_len);
    return PP_OK;
}
