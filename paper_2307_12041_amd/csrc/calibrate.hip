// calibrate.hip -- the matrix-core calibration hook of include/pplace.h: a kernel that does nothing
// but bf16 MFMAs on normally distributed operands, so that timing it gives the rate the matrix cores
// sustain on data like the contractions' operands when every CU is loaded (the clock under such a
// load is set by the power limit, not by the instruction rate, and it depends on the operand bits:
// zeros draw far less power than random mantissas).  It computes nothing of the method.
#include "../../include/pplace.h"
#include "common.h"

namespace pp {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// A standard normal value from a 32-bit counter: two uniforms from the PCG output hash of the
// counter and of its golden-ratio offset, then the Box-Muller transform.
__device__ __forceinline__ unsigned pcg_hash(unsigned x) {
    x = x * 747796405u + 2891336453u;
    x = ((x >> ((x >> 28) + 4u)) ^ x) * 277803737u;
    return (x >> 22) ^ x;
}
__device__ __forceinline__ float normal_from(unsigned ctr) {
    const float u1 = (float)(pcg_hash(ctr) >> 8) * (1.0f / 16777216.0f) + 0x1p-25f;
    const float u2 = (float)(pcg_hash(ctr ^ 0x9e3779b9u) >> 8) * (1.0f / 16777216.0f);
    return sqrtf(-2.0f * logf(u1)) * cospif(2.0f * u2);
}

// Each wave: four A and four B operand sets, 16 accumulator tiles, 16 MFMAs per iteration (A set
// m % 4, B set m / 4 for tile m), nothing else in the loop.
__global__ __launch_bounds__(256) void k_mfma_calibrate(float *__restrict__ out, int iters) {
    const unsigned tid = threadIdx.x, wg = blockIdx.x;
    bf16x8 A[4], B[4];
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const unsigned c = ((wg * 256u + tid) * 4u + (unsigned)q) * 16u + (unsigned)i;
            A[q][i] = (__bf16)normal_from(2u * c);
            B[q][i] = (__bf16)normal_from(2u * c + 1u);
        }
    f32x16 acc[16];
#pragma unroll
    for (int m = 0; m < 16; ++m)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[m][r] = 0.0f;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int m = 0; m < 16; ++m)
            acc[m] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A[m & 3], B[m >> 2], acc[m], 0, 0, 0);
    }
    float s = 0.0f;
#pragma unroll
    for (int m = 0; m < 16; ++m)
#pragma unroll
        for (int r = 0; r < 16; ++r) s += acc[m][r];
    out[(size_t)wg * 256 + tid] = s;
}

}  // namespace
}  // namespace pp

extern "C" int pp_mfma_calibrate(int workgroups, int iters, float *out, void *stream) {
    if (workgroups < 1 || workgroups > 65535 || iters < 1 || out == nullptr) return PP_ERR_ARG;
    hipLaunchKernelGGL(pp::k_mfma_calibrate, dim3(workgroups), dim3(256), 0, (hipStream_t)stream, out, iters);
    return hipGetLastError() == hipSuccess ? PP_OK : PP_ERR_DEVICE;
}
