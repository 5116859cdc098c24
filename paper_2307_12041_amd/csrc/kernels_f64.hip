// kernels_f64.hip -- FP64 and FP32 paths: basis tiles generated on chip in FP64 (rounded to the
// operand type when stored), contractions on v_mfma_f64_16x16x4 (FP64) or v_mfma_f32_16x16x4 (FP32).
//
// Forward (coefficients, Sec. III-A closed forms): At[u][p] = sum_i S_iu T_ip over a K range of
// blocks, one FP64 partial per split.  Backward (field of eq. ksi integrated over each block):
// G[i][n] = sum_k A_ik B[k][n] with the sine-difference basis A generated along the K frequency
// axis, then the row dot  g_i = sum_n E_in G[i][n]  with the cosine-difference basis E.
//
// Lane layouts (16x16 output, K = 4, one value per lane for A and B): A[i][k] in lane i + 16k and
// B[k][j] in lane j + 16k for both; the output differs:
//   v_mfma_f64_16x16x4: D[i][j] in lane j + 16 (i % 4), element i / 4;
//   v_mfma_f32_16x16x4: D[i][j] in lane j + 16 (i / 4), element i % 4.
//
// Basis generation: for a block edge e and frequency k, the phase k*pi*e/L is carried in half
// turns.  A run of consecutive frequencies starts from an FP64 seed, reduced to [-1, 1] half
// turns before sincospi, and continues by rotating the (cos, sin) pair by the one-step phasor.
// Runs are at most 32 long, so the rotation error stays at a few ulp.
#include <type_traits>

#include "common.h"

namespace pp {
namespace {

// Operand type T: the MFMA and its output row for (lane, element).
template <typename T> struct Mat;
template <> struct Mat<double> {
    typedef double v4 __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ v4 mfma(double a, double b, v4 c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int r) { return 4 * r + (lane >> 4); }
};
template <> struct Mat<float> {
    typedef float v4 __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ v4 mfma(float a, float b, v4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

__device__ __forceinline__ double reduce_half_turns(double t) { return t - 2.0 * rint(0.5 * t); }

struct EdgeRot {
    double cp, sp, cm, sm;      // current phasors of the + and - edges
    double c1p, s1p, c1m, s1m;  // one-frequency-step phasors
    __device__ __forceinline__ void init(double c, double sz, double L, int k0) {
        const double tp = (c + 0.5 * sz) / L;
        const double tm = (c - 0.5 * sz) / L;
        sincospi(reduce_half_turns((double)k0 * tp), &sp, &cp);
        sincospi(reduce_half_turns((double)k0 * tm), &sm, &cm);
        sincospi(reduce_half_turns(tp), &s1p, &c1p);
        sincospi(reduce_half_turns(tm), &s1m, &c1m);
    }
    __device__ __forceinline__ void step() {
        double t = cp * c1p - sp * s1p;
        sp = sp * c1p + cp * s1p;
        cp = t;
        t = cm * c1m - sm * s1m;
        sm = sm * c1m + cm * s1m;
        cm = t;
    }
};

// One phasor of a point (centre) coordinate: cos and sin of w_k c for consecutive k.
struct PointRot {
    double c, s, c1, s1;
    __device__ __forceinline__ void init(double x, double L, int k0) {
        const double t = x / L;
        sincospi(reduce_half_turns((double)k0 * t), &s, &c);
        sincospi(reduce_half_turns(t), &s1, &c1);
    }
    __device__ __forceinline__ void step() {
        const double t = c * c1 - s * s1;
        s = s * c1 + c * s1;
        c = t;
    }
};

// R consecutive values of one kind (RunKind) for one block, written at dst[k*stride] (generated in FP64,
// rounded to T when stored).
template <int KIND, int R, typename T>
__device__ __forceinline__ void gen_run(double c, double sz, double L, int k0, bool valid, T *dst, int stride) {
    if (!valid) {
#pragma unroll
        for (int k = 0; k < R; ++k) dst[k * stride] = (T)0;
        return;
    }
    if constexpr (KIND == RUN_SINDIFF || KIND == RUN_COSDIFF) {
        EdgeRot r;
        r.init(c, sz, L, k0);
#pragma unroll
        for (int k = 0; k < R; ++k) {
            if constexpr (KIND == RUN_SINDIFF)
                dst[k * stride] = (T)((k0 + k == 0) ? sz : (r.sp - r.sm));
            else
                dst[k * stride] = (T)(r.cp - r.cm);
            r.step();
        }
    } else {
        PointRot r;
        r.init(c, L, k0);
        const double pil = kPi / L;
#pragma unroll
        for (int k = 0; k < R; ++k) {
            if constexpr (KIND == RUN_COS)
                dst[k * stride] = (T)r.c;
            else
                dst[k * stride] = (T)((double)(k0 + k) * pil * r.s);
            r.step();
        }
    }
}

// A run of R consecutive frequencies of one block that moves on by J frequencies every K chunk (the
// row-form contraction, where a thread keeps its block for the whole K loop), for the K-side kinds
// RUN_SINDIFF (the product form 2 cos(k a) sin(k b), a = pi c / L, b = pi size / (2L)) and RUN_COS
// (cos(k a), a = pi c / L).  The phasors e^{i k0 a} (and e^{i k0 b}) at the run's first frequency,
// the one-frequency step and the J-frequency jump come from FP64 sincospi of exactly reduced
// arguments once; each run is then produced by the three-term recurrence f_{k+1} = 2 cos(t) f_k -
// f_{k-1} of each factor, and after each chunk the seed phasors are rotated by the jump instead of
// being evaluated again.
template <int KIND>
struct KRun {
    static_assert(KIND == RUN_SINDIFF || KIND == RUN_COS, "K-side kinds of the row-form contraction");
    static constexpr bool kProd = KIND == RUN_SINDIFF;
    double ca, sa, cb, sb;        // seed phasors at the run's first frequency (b: RUN_SINDIFF only)
    double c1a, s1a, c1b, s1b;    // one-frequency step
    double cja, sja, cjb, sjb;    // J-frequency jump
    double sz;

    __device__ __forceinline__ void init(double c, double size, double L, int k0, int J) {
        sz = size;
        const double ta = c / L;
        sincospi(reduce_half_turns((double)k0 * ta), &sa, &ca);
        sincospi(reduce_half_turns(ta), &s1a, &c1a);
        sincospi(reduce_half_turns((double)J * ta), &sja, &cja);
        if constexpr (kProd) {
            const double tb = 0.5 * size / L;
            sincospi(reduce_half_turns((double)k0 * tb), &sb, &cb);
            sincospi(reduce_half_turns(tb), &s1b, &c1b);
            sincospi(reduce_half_turns((double)J * tb), &sjb, &cjb);
        }
    }

    // The R values at frequencies k0 .. k0 + R - 1, written at dst[k * stride] (rounded to T).
    template <int R, typename T>
    __device__ __forceinline__ void gen(int k0, bool valid, T *dst, int stride) const {
        if (!valid) {
#pragma unroll
            for (int k = 0; k < R; ++k) dst[k * stride] = (T)0;
            return;
        }
        double C = ca, Cm = ca * c1a + sa * s1a;                  // cos(k0 a), cos((k0 - 1) a)
        const double ta2 = 2.0 * c1a;
        double S = 0.0, Sm = 0.0, tb2 = 0.0;
        if constexpr (kProd) {
            S = 2.0 * sb;                                         // 2 sin(k0 b), 2 sin((k0 - 1) b)
            Sm = 2.0 * (sb * c1b - cb * s1b);
            tb2 = 2.0 * c1b;
        }
#pragma unroll
        for (int k = 0; k < R; ++k) {
            if constexpr (kProd)
                dst[k * stride] = (T)((k0 + k == 0) ? sz : C * S);
            else
                dst[k * stride] = (T)C;
            const double Cn = fma(ta2, C, -Cm);
            Cm = C;
            C = Cn;
            if constexpr (kProd) {
                const double Sn = fma(tb2, S, -Sm);
                Sm = S;
                S = Sn;
            }
        }
    }

    __device__ __forceinline__ void jump() {
        const double t = ca * cja - sa * sja;
        sa = sa * cja + ca * sja;
        ca = t;
        if constexpr (kProd) {
            const double u = cb * cjb - sb * sjb;
            sb = sb * cjb + cb * sjb;
            cb = u;
        }
    }
};

// R consecutive sine-difference integrals S_k = sin(w_k x+) - sin(w_k x-) of one block (S_0 = its
// size), k = k0 .. k0 + R - 1, in the product form 2 cos(k a) sin(k b), a = pi c / L,
// b = pi size / (2L), each factor by its three-term recurrence f_{k+1} = 2 cos(t) f_k - f_{k-1}
// from FP64 seeds at k0 and k0 - 1: two FMAs and one product per value (two phasor rotations cost
// eight), with no cancellation for narrow blocks.  Written at dst[k * stride], rounded to T.
template <int R, typename T>
__device__ __forceinline__ void gen_sindiff(double c, double sz, double L, int k0, bool valid, T *dst, int stride) {
    if (!valid) {
#pragma unroll
        for (int k = 0; k < R; ++k) dst[k * stride] = (T)0;
        return;
    }
    const double ta = c / L, tb = 0.5 * sz / L;
    double sa, ca, s1a, c1a, sb, cb, s1b, c1b;
    sincospi(reduce_half_turns((double)k0 * ta), &sa, &ca);
    sincospi(reduce_half_turns(ta), &s1a, &c1a);
    sincospi(reduce_half_turns((double)k0 * tb), &sb, &cb);
    sincospi(reduce_half_turns(tb), &s1b, &c1b);
    double C = ca, Cm = ca * c1a + sa * s1a;                  // cos(k0 a), cos((k0 - 1) a)
    double S = 2.0 * sb, Sm = 2.0 * (sb * c1b - cb * s1b);    // 2 sin(k0 b), 2 sin((k0 - 1) b)
    const double ta2 = 2.0 * c1a, tb2 = 2.0 * c1b;
#pragma unroll
    for (int k = 0; k < R; ++k) {
        dst[k * stride] = (T)((k0 + k == 0) ? sz : C * S);
        const double Cn = fma(ta2, C, -Cm);
        Cm = C;
        C = Cn;
        const double Sn = fma(tb2, S, -Sm);
        Sm = S;
        S = Sn;
    }
}

// ------------------------------------------------------------------------------------------------
// Forward: grid (tiles_u * tiles_p, splits), 256 threads as 2 x 2 waves over a TU x TP tile.
// LDS holds the K chunk of the two basis tiles, k-major: Xs[kb][u], Ys[kb][p].
// ------------------------------------------------------------------------------------------------
template <typename T, int TU, int TP, int KB>
__global__ __launch_bounds__(256) void k_fwd_mat(int64_t n, int Mu, int Mp, double W, double H,
                                                 const double *__restrict__ x, const double *__restrict__ y,
                                                 const double *__restrict__ w, const double *__restrict__ h,
                                                 T *__restrict__ part, int tiles_p, int64_t chunks,
                                                 int64_t chunks_per_split) {
    typedef typename Mat<T>::v4 v4;
    constexpr int LU = TU + 1, LP = TP + 1;
    __shared__ T Xs[KB * LU];
    __shared__ T Ys[KB * LP];
    constexpr int WU = TU / 2, WP = TP / 2, SU = WU / 16, SP = WP / 16;
    constexpr int RX = TU * KB / 128, RY = TP * KB / 128;
    static_assert(RX * 128 == TU * KB && RY * 128 == TP * KB, "tile/thread mismatch");

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int tu0 = (int)(blockIdx.x / tiles_p) * TU, tp0 = (int)(blockIdx.x % tiles_p) * TP;
    const int wu0 = (wave >> 1) * WU, wp0 = (wave & 1) * WP;
    const int64_t c_begin = (int64_t)blockIdx.y * chunks_per_split;
    const int64_t c_end = min(chunks, c_begin + chunks_per_split);

    const int side = tid >> 7, j = tid & 127, kb = j % KB, run = j / KB;

    v4 acc[SU][SP];
#pragma unroll
    for (int a = 0; a < SU; ++a)
#pragma unroll
        for (int b = 0; b < SP; ++b) acc[a][b] = v4{(T)0, (T)0, (T)0, (T)0};

    for (int64_t c = c_begin; c < c_end; ++c) {
        const int64_t ib = c * KB + kb;
        const bool valid = ib < n;
        __syncthreads();
        if (side == 0) {
            const double cx = valid ? x[ib] : 0.0, sx = valid ? w[ib] : 0.0;
            gen_sindiff<RX>(cx, sx, W, tu0 + run * RX, valid, &Xs[kb * LU + run * RX], 1);
        } else {
            const double cy = valid ? y[ib] : 0.0, sy = valid ? h[ib] : 0.0;
            gen_sindiff<RY>(cy, sy, H, tp0 + run * RY, valid, &Ys[kb * LP + run * RY], 1);
        }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < KB / 4; ++ks) {
            const int kr = ks * 4 + (lane >> 4);
            T av[SU], bv[SP];
#pragma unroll
            for (int a = 0; a < SU; ++a) av[a] = Xs[kr * LU + wu0 + a * 16 + (lane & 15)];
#pragma unroll
            for (int b = 0; b < SP; ++b) bv[b] = Ys[kr * LP + wp0 + b * 16 + (lane & 15)];
#pragma unroll
            for (int a = 0; a < SU; ++a)
#pragma unroll
                for (int b = 0; b < SP; ++b) acc[a][b] = Mat<T>::mfma(av[a], bv[b], acc[a][b]);
        }
    }

    T *out = part + (size_t)blockIdx.y * (size_t)Mu * (size_t)Mp;
#pragma unroll
    for (int a = 0; a < SU; ++a)
#pragma unroll
        for (int b = 0; b < SP; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int u = tu0 + wu0 + a * 16 + Mat<T>::row(lane, r);
                const int p = tp0 + wp0 + b * 16 + (lane & 15);
                if (u < Mu && p < Mp) out[(size_t)u * Mp + p] = acc[a][b][r];
            }
}

// ------------------------------------------------------------------------------------------------
// Row-form contraction (the backward and the evaluation entry points): for each block (or point)
// i of a TB tile and each epilogue frequency j of a TN tile,
//     Z_ij = sum_k Bas_ik B[k][j]          (K loop over the Ka frequencies of one axis, MFMA),
//     out_i += sum_j E_ij Z_ij             (fused row-dot epilogue, FP64),
// with Bas of kind KK_KIND along the K axis and E of kind EP1 (and, if EP2 >= 0, a second
// epilogue of kind EP2 on the same Z into gpart2).  Grid (tiles_b, tiles_n), 256 threads as 2 x 2
// waves.  LDS: As[k][i] (generated basis), Bs[k][j] (prepared operand); after the K loop the same
// space holds the epilogue basis of one half of the N tile, Es[j][i].  Two waves per SIMD (at most
// 256 registers per lane; FP64 fits without spills): the LDS (68 KB in FP64) admits two workgroups
// per CU, so one workgroup's MFMAs run while the other generates its next basis chunk and loads
// its next operand chunk, which sit between barriers.
// ------------------------------------------------------------------------------------------------
template <typename T, int TB, int TN, int KK, int KA_KIND, int EP1, int EP2>
__global__ __launch_bounds__(256, 2) void k_bwd_mat(int64_t n, BwdAxis ax) {
    typedef typename Mat<T>::v4 v4;
    constexpr int LB = TB + 1, LN = TN + 1;
    constexpr int HALF = TN / 2;
    static_assert(TB == 128 && TN == 128 && KK == 32, "LDS reuse below assumes this tile");
    constexpr int SMEM = (KK * LB + KK * LN) > (HALF * LB) ? (KK * LB + KK * LN) : (HALF * LB);
    __shared__ T smem[SMEM];
    __shared__ double red[2 * TB];
    T *As = smem, *Bs = smem + KK * LB, *Es = smem;
    constexpr int WI = TB / 2, WJ = TN / 2, SI = WI / 16, SJ = WJ / 16;
    constexpr int RA = KK * TB / 256;   // K-side run per thread per chunk
    constexpr int RE = HALF * TB / 256; // epilogue run per thread per half

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t ib0 = (int64_t)blockIdx.x * TB;
    const int n0 = (int)blockIdx.y * TN;
    const int wi0 = (wave >> 1) * WI, wc = wave & 1, wj0 = wc * WJ;
    const int gi = tid % TB, grun = tid / TB;
    const int64_t ib = ib0 + gi;
    const bool valid = ib < n;
    const double ca = valid ? ax.ca[ib] : 0.0, sa = (valid && ax.sa) ? ax.sa[ib] : 0.0;
    const double cb = valid ? ax.cb[ib] : 0.0, sb = (valid && ax.sb) ? ax.sb[ib] : 0.0;
    const T *__restrict__ B = (const T *)ax.B;

    v4 acc[SI][SJ];
#pragma unroll
    for (int a = 0; a < SI; ++a)
#pragma unroll
        for (int b = 0; b < SJ; ++b) acc[a][b] = v4{(T)0, (T)0, (T)0, (T)0};

    KRun<KA_KIND> krun{};
    if (valid) krun.init(ca, sa, ax.La, grun * RA, KK);
    constexpr int PB = KK * TN / 256;
    for (int k0 = 0; k0 < ax.Ka; k0 += KK) {
        // The operand chunk is loaded first (unconditionally, from a valid address; the bounds are
        // applied when it is stored), so that its latency overlaps the basis generation.
        T bv[PB];
#pragma unroll
        for (int q = 0; q < PB; ++q) {
            const int idx = tid + 256 * q, k = idx / TN, jj = idx % TN;
            const bool in = (k0 + k < ax.Ka) && (n0 + jj < ax.Nb);
            bv[q] = B[in ? (size_t)(k0 + k) * ax.Nb + n0 + jj : 0];
        }
        __syncthreads();
        krun.template gen<RA>(k0 + grun * RA, valid, &As[(grun * RA) * LB + gi], LB);
        krun.jump();
#pragma unroll
        for (int q = 0; q < PB; ++q) {
            const int idx = tid + 256 * q, k = idx / TN, jj = idx % TN;
            const bool in = (k0 + k < ax.Ka) && (n0 + jj < ax.Nb);
            Bs[k * LN + jj] = in ? bv[q] : (T)0;
        }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < KK / 4; ++ks) {
            const int kr = ks * 4 + (lane >> 4);
            T av[SI], bv[SJ];
#pragma unroll
            for (int a = 0; a < SI; ++a) av[a] = As[kr * LB + wi0 + a * 16 + (lane & 15)];
#pragma unroll
            for (int b = 0; b < SJ; ++b) bv[b] = Bs[kr * LN + wj0 + b * 16 + (lane & 15)];
#pragma unroll
            for (int a = 0; a < SI; ++a)
#pragma unroll
                for (int b = 0; b < SJ; ++b) acc[a][b] = Mat<T>::mfma(av[a], bv[b], acc[a][b]);
        }
    }

    // Epilogue(s): row dot with the epilogue basis, one N half at a time; the 16 lanes that share
    // a row are summed by a fixed butterfly, the two column waves in fixed order.
    auto epilogue = [&](auto kind_tag, double *__restrict__ gpart) {
        constexpr int EK = decltype(kind_tag)::value;
        double rs[SI][4];
#pragma unroll
        for (int a = 0; a < SI; ++a)
#pragma unroll
            for (int r = 0; r < 4; ++r) rs[a][r] = 0.0;
        for (int hf = 0; hf < 2; ++hf) {
            __syncthreads();
            gen_run<EK, RE>(cb, sb, ax.Lb, n0 + hf * HALF + grun * RE, valid, &Es[(grun * RE) * LB + gi], LB);
            __syncthreads();
            if (wc == hf) {
#pragma unroll
                for (int a = 0; a < SI; ++a)
#pragma unroll
                    for (int b = 0; b < SJ; ++b)
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            const int il = wi0 + a * 16 + Mat<T>::row(lane, r);
                            const int jl = b * 16 + (lane & 15);
                            rs[a][r] += (double)acc[a][b][r] * (double)Es[jl * LB + il];
                        }
            }
        }
#pragma unroll
        for (int a = 0; a < SI; ++a)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                double v = rs[a][r];
                v += __shfl_xor(v, 1);
                v += __shfl_xor(v, 2);
                v += __shfl_xor(v, 4);
                v += __shfl_xor(v, 8);
                rs[a][r] = v;
            }
        if ((lane & 15) == 0) {
#pragma unroll
            for (int a = 0; a < SI; ++a)
#pragma unroll
                for (int r = 0; r < 4; ++r) red[wc * TB + wi0 + a * 16 + Mat<T>::row(lane, r)] = rs[a][r];
        }
        __syncthreads();
        if (tid < TB && ib0 + tid < n)
            gpart[(size_t)blockIdx.y * (size_t)n + (size_t)(ib0 + tid)] = red[tid] + red[TB + tid];
    };
    epilogue(std::integral_constant<int, EP1>{}, ax.gpart);
    if constexpr (EP2 >= 0) epilogue(std::integral_constant<int, (EP2 >= 0 ? EP2 : 0)>{}, ax.gpart2);
}

template <typename T>
hipError_t launch_fwd_mat(const FwdPlan &pl, int64_t n, int Mu, int Mp, double W, double H, const double *x,
                          const double *y, const double *w, const double *h, T *part, hipStream_t s) {
    dim3 grid(pl.tiles_u * pl.tiles_p, pl.splits);
    if (pl.tu == 128 && pl.tp == 128 && pl.kb == 32)
        hipLaunchKernelGGL((k_fwd_mat<T, 128, 128, 32>), grid, dim3(256), 0, s, n, Mu, Mp, W, H, x, y, w, h, part,
                           pl.tiles_p, pl.chunks, pl.chunks_per_split);
    else if (pl.tu == 64 && pl.tp == 64 && pl.kb == 32)
        hipLaunchKernelGGL((k_fwd_mat<T, 64, 64, 32>), grid, dim3(256), 0, s, n, Mu, Mp, W, H, x, y, w, h, part,
                           pl.tiles_p, pl.chunks, pl.chunks_per_split);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

template <typename T, int KA_KIND, int EP1, int EP2>
hipError_t launch_rowform(const BwdPlan &pl, int64_t n, const BwdAxis &ax, hipStream_t s) {
    if (!(pl.tb == 128 && pl.tn == 128 && pl.kk == 32)) return hipErrorInvalidValue;
    if (n == 0) return hipSuccess;
    const int tiles_n = (ax.Nb + pl.tn - 1) / pl.tn;
    const int64_t tiles_b = (n + pl.tb - 1) / pl.tb;
    dim3 grid((unsigned)tiles_b, tiles_n);
    hipLaunchKernelGGL((k_bwd_mat<T, 128, 128, 32, KA_KIND, EP1, EP2>), grid, dim3(256), 0, s, n, ax);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_rowform_kind(RowForm f, const BwdPlan &pl, int64_t n, const BwdAxis &ax, hipStream_t s) {
    switch (f) {
        case ROW_FIELD: return launch_rowform<T, RUN_SINDIFF, RUN_COSDIFF, -1>(pl, n, ax, s);
        case ROW_POTENTIAL: return launch_rowform<T, RUN_SINDIFF, RUN_SINDIFF, -1>(pl, n, ax, s);
        case ROW_POINT_DUAL: return launch_rowform<T, RUN_COS, RUN_COS, RUN_WSIN>(pl, n, ax, s);
        case ROW_POINT_WSIN: return launch_rowform<T, RUN_COS, RUN_WSIN, -1>(pl, n, ax, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_fwd_f64(const FwdPlan &pl, int64_t n, int Mu, int Mp, double W, double H, const double *x,
                          const double *y, const double *w, const double *h, double *part, hipStream_t s) {
    return launch_fwd_mat<double>(pl, n, Mu, Mp, W, H, x, y, w, h, part, s);
}
hipError_t launch_fwd_f32(const FwdPlan &pl, int64_t n, int Mu, int Mp, double W, double H, const double *x,
                          const double *y, const double *w, const double *h, float *part, hipStream_t s) {
    return launch_fwd_mat<float>(pl, n, Mu, Mp, W, H, x, y, w, h, part, s);
}
hipError_t launch_rowform_f64(RowForm f, const BwdPlan &pl, int64_t n, const BwdAxis &ax, hipStream_t s) {
    return launch_rowform_kind<double>(f, pl, n, ax, s);
}
hipError_t launch_rowform_f32(RowForm f, const BwdPlan &pl, int64_t n, const BwdAxis &ax, hipStream_t s) {
    return launch_rowform_kind<float>(f, pl, n, ax, s);
}

}  // namespace pp
