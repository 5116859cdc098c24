// kernels_common.hip -- precision-independent FP64 stages: split-K reduction + spectral scale +
// energy partials, the final energy sum, backward operand preparation, and the final per-block
// gradient sum.  Every reduction runs in a fixed order, so results are bitwise reproducible.
#include "common.h"

namespace pp {
namespace {

constexpr int kRedThreads = 256;

// Deterministic block sum of one double per thread (butterfly inside waves, then wave order).
__device__ __forceinline__ double block_sum(double v, double *scratch) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) scratch[wave] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int k = 0; k < (int)(blockDim.x >> 6); ++k) s += scratch[k];
    return s;  // valid in thread 0
}

// Coefficients from the split-K partial contractions At = sum_s part[s]:
//   A_up = At_up / (wt_u vt_p),   a_up = s_up A_up,
//   s_up = e_u e_p / (W H (w_u^2 + v_p^2)), e_0 = 1, e_k = 2, s_00 = 0
// (the four coefficient cases of Sec. III-A written with one scale; a_00 = 0 is the
// compatibility condition).  The energy partial of this block is sum a_up A_up.
__global__ __launch_bounds__(kRedThreads) void k_reduce_scale(const void *__restrict__ part, int part_f32,
                                                              int splits, int Mu, int Mp, double W, double H,
                                                              double *__restrict__ a, double *__restrict__ epart) {
    __shared__ double scratch[kRedThreads / 64];
    const size_t MM = (size_t)Mu * (size_t)Mp;
    const size_t idx = (size_t)blockIdx.x * kRedThreads + threadIdx.x;
    double e = 0.0;
    if (idx < MM) {
        const int u = (int)(idx / (size_t)Mp), p = (int)(idx % (size_t)Mp);
        double At = 0.0;
        if (part_f32) {
            const float *pf = (const float *)part;
            for (int s = 0; s < splits; ++s) At += (double)pf[(size_t)s * MM + idx];
        } else {
            const double *pd = (const double *)part;
            for (int s = 0; s < splits; ++s) At += pd[(size_t)s * MM + idx];
        }
        const double wu = (double)u * kPi / W, vp = (double)p * kPi / H;
        const double wt = u ? wu : 1.0, vt = p ? vp : 1.0;
        const double A = At / (wt * vt);
        const double eps = (u ? 2.0 : 1.0) * (p ? 2.0 : 1.0);
        const double sc = (u == 0 && p == 0) ? 0.0 : eps / (W * H * (wu * wu + vp * vp));
        const double av = sc * A;
        if (a) a[idx] = av;
        e = av * A;
    }
    const double s = block_sum(e, scratch);
    if (threadIdx.x == 0) epart[blockIdx.x] = s;
}

__global__ __launch_bounds__(kRedThreads) void k_energy_final(const double *__restrict__ epart, int nb,
                                                              double *__restrict__ E) {
    __shared__ double scratch[kRedThreads / 64];
    double v = 0.0;
    for (int k = threadIdx.x; k < nb; k += kRedThreads) v += epart[k];
    const double s = block_sum(v, scratch);
    if (threadIdx.x == 0) *E = 0.5 * s;
}

// Operands of the row-form contractions: BxT[p][u] (K = p, epilogue over u) and By[u][p] (K = u,
// epilogue over p), a times the frequency factors of the chosen form.
template <typename T>
__global__ void k_prep_rowform(int form, const double *__restrict__ a, int Mu, int Mp, double W, double H,
                               T *__restrict__ BxT, T *__restrict__ By) {
    const size_t MM = (size_t)Mu * (size_t)Mp;
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= MM) return;
    const int u = (int)(idx / (size_t)Mp), p = (int)(idx % (size_t)Mp);
    const double wt = u ? (double)u * kPi / W : 1.0, vt = p ? (double)p * kPi / H : 1.0;
    const double av = a[idx];
    double bx = av, by = av;
    if (form == ROW_FIELD) {
        bx = av / vt;
        by = av / wt;
    } else if (form == ROW_POTENTIAL) {
        bx = av / (vt * wt);
    }
    if (BxT) BxT[(size_t)p * Mu + u] = (T)bx;
    if (By) By[idx] = (T)by;
}

__global__ void k_bwd_final(const double *__restrict__ gpx, int tx, const double *__restrict__ gpy, int ty,
                            int64_t n, const double *__restrict__ dE, double *__restrict__ gx,
                            double *__restrict__ gy) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double d = dE ? *dE : 1.0;
    if (gx) {
        double sx = 0.0;
        for (int t = 0; t < tx; ++t) sx += gpx[(size_t)t * n + i];
        gx[i] = d * sx;
    }
    if (gy) {
        double sy = 0.0;
        for (int t = 0; t < ty; ++t) sy += gpy[(size_t)t * n + i];
        gy[i] = d * sy;
    }
}

}  // namespace

int reduce_scale_blocks(int Mu, int Mp) {
    const size_t MM = (size_t)Mu * (size_t)Mp;
    return (int)((MM + kRedThreads - 1) / kRedThreads);
}

hipError_t launch_reduce_scale(const void *part, bool part_f32, int splits, int Mu, int Mp, double W, double H,
                               double *a, double *epart, int *nblocks_out, hipStream_t s) {
    const int nb = reduce_scale_blocks(Mu, Mp);
    hipLaunchKernelGGL(k_reduce_scale, dim3(nb), dim3(kRedThreads), 0, s, part, part_f32 ? 1 : 0, splits, Mu, Mp,
                       W, H, a, epart);
    if (nblocks_out) *nblocks_out = nb;
    return hipGetLastError();
}

hipError_t launch_energy_final(const double *epart, int nblocks, double *E, hipStream_t s) {
    hipLaunchKernelGGL(k_energy_final, dim3(1), dim3(kRedThreads), 0, s, epart, nblocks, E);
    return hipGetLastError();
}

hipError_t launch_prep_rowform_f64(RowForm f, const double *a, int Mu, int Mp, double W, double H, double *BxT,
                                   double *By, hipStream_t s) {
    const size_t MM = (size_t)Mu * (size_t)Mp;
    hipLaunchKernelGGL(k_prep_rowform<double>, dim3((unsigned)((MM + 255) / 256)), dim3(256), 0, s, (int)f, a, Mu,
                       Mp, W, H, BxT, By);
    return hipGetLastError();
}

hipError_t launch_prep_rowform_f32(RowForm f, const double *a, int Mu, int Mp, double W, double H, float *BxT,
                                   float *By, hipStream_t s) {
    const size_t MM = (size_t)Mu * (size_t)Mp;
    hipLaunchKernelGGL(k_prep_rowform<float>, dim3((unsigned)((MM + 255) / 256)), dim3(256), 0, s, (int)f, a, Mu,
                       Mp, W, H, BxT, By);
    return hipGetLastError();
}

hipError_t launch_bwd_final(const double *gpx, int tx, const double *gpy, int ty, int64_t n, const double *dE,
                            double *gx, double *gy, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_bwd_final, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, gpx, tx, gpy, ty, n, dE, gx,
                       gy);
    return hipGetLastError();
}

}  // namespace pp
