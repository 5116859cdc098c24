// kernels_bf16.hip -- BF16 hi/lo split path (PP_BF16X3) and plain BF16 (PP_BF16): basis values
// generated in FP32 on chip, split into bf16 hi + lo, contracted on v_mfma_f32_32x32x16_bf16 with
// FP32 accumulation (x3: hi*hi + hi*lo + lo*hi).
//
// Basis in product form (no cancellation for narrow blocks): for a block of centre c and size sz
// on an axis of length L, alpha = pi c / L, beta = pi sz / (2L), and frequency k >= 1,
//     S_k = sin(k (alpha + beta)) - sin(k (alpha - beta)) = 2 cos(k alpha) sin(k beta),
//     K_k = cos(k (alpha + beta)) - cos(k (alpha - beta)) = -2 sin(k alpha) sin(k beta),
// with S_0 = sz, K_0 = 0 (the sine- and cosine-difference factors of the closed-form
// coefficients, Sec. III-A, and of the field, eq. ksi).  Runs of consecutive frequencies start
// from FP64-reduced seeds and continue by the three-term recurrence
//     f_{k+1} = 2 cos(theta) f_k - f_{k-1},
// whose coefficient 2 cos(theta) is carried as an fp32 hi + lo pair so that the frequency is
// exact to ~1e-14 even for theta near 0 or pi; runs are at most 32 long (error <~ 1e-5).
//
// Lane layout of v_mfma_f32_32x32x16_bf16 (wave64): A[i][k] with i = lane % 32 and
// k = 8 (lane / 32) + e (e = 0..7 in the operand vector); B[k][j] with j = lane % 32 and the same
// k; D[i][j] in lane j + 32 (i / 4 % 2), element 4 (i / 8) + i % 4.
//
// LDS transpose read ds_read_b64_tr_b16 (per group of 16 lanes): result lane i, element j is
// element i % 4 of the 64 bits addressed by source lane 4 j + i / 4.
#include "common.h"

namespace pp {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef short s16x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned u32x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ double reduce_half_turns(double t) { return t - 2.0 * rint(0.5 * t); }

// cos/sin of pi*(k*t) for integer k, with the product reduced in FP64.
__device__ __forceinline__ void seed_phasor(int k, double t, float &c, float &s) {
    const float r = (float)reduce_half_turns((double)k * t);
    sincospif(r, &s, &c);
}

__device__ __forceinline__ unsigned pack_bf16(float a, float b) {
    bf16x2 v = {(__bf16)a, (__bf16)b};
    return __builtin_bit_cast(unsigned, v);
}

// Split two fp32 values into packed bf16 hi (round to nearest even) and packed bf16 lo of the
// remainders.
__device__ __forceinline__ void split2(float a, float b, unsigned &hi, unsigned &lo) {
    hi = pack_bf16(a, b);
    const float ha = __builtin_bit_cast(float, hi << 16);
    const float hb = __builtin_bit_cast(float, hi & 0xffff0000u);
    lo = pack_bf16(a - ha, b - hb);
}

// Three-term recurrence state for cos(k alpha) (or any sinusoid) with a hi/lo coefficient.
struct Cheb {
    float f, fm, ch, cl;  // f_k, f_{k-1}, 2cos(theta) = ch + cl
    __device__ __forceinline__ float next() {
        const float nx = fmaf(ch, f, fmaf(cl, f, -fm));
        fm = f;
        f = nx;
        return nx;
    }
};

}  // namespace

// Per-block phase record for one axis (see common.h).
__global__ void k_phase_table(int64_t n, const double *__restrict__ c, const double *__restrict__ sz, double L,
                              PhaseRec *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double ta = c[i] / L, tb = sz[i] / (2.0 * L);
    PhaseRec r;
    r.ta = ta;
    r.tb = tb;
    double s, co;
    sincospi(reduce_half_turns(ta), &s, &co);
    r.ca = (float)co; r.sa = (float)s;
    r.c2ah = (float)(2.0 * co); r.c2al = (float)(2.0 * co - (double)r.c2ah);
    sincospi(reduce_half_turns(tb), &s, &co);
    r.cb = (float)co; r.sb = (float)s;
    r.c2bh = (float)(2.0 * co); r.c2bl = (float)(2.0 * co - (double)r.c2bh);
    sincospi(reduce_half_turns(32.0 * ta), &s, &co);
    r.ca32 = (float)co; r.sa32 = (float)s;
    sincospi(reduce_half_turns(32.0 * tb), &s, &co);
    r.cb32 = (float)co; r.sb32 = (float)s;
    r.size = (float)sz[i];
    r.pad0 = r.pad1 = r.pad2 = 0.0f;
    out[i] = r;
}

namespace {

// ================================================================================================
// Forward: At[u][p] = sum_i S_iu T_ip over a range of blocks.
// 512 threads = 8 waves in two ping-pong groups.  Wave w owns the 128 x 64 output sub-tile
// (u-half w / 4, p-quarter w % 4); waves w and w + 4 share a SIMD.  Per chunk of 32 blocks the
// group of waves 0-3 generates the X tile, the group of waves 4-7 the Y tile; while one group
// contracts chunk c from one LDS buffer the other generates chunk c + 1 into the other buffer.
// LDS tile layout: [block][frequency] bf16, rows padded to 544 bytes; MFMA operands are read
// with the transpose read.
// ================================================================================================
constexpr int FT = 256;              // output tile (u and p)
constexpr int FKB = 32;              // blocks per chunk
constexpr int FROW = FT * 2 + 32;    // bytes per LDS row
constexpr int FARR = FKB * FROW;     // bytes per array
constexpr int FBUF = 4 * FARR;       // Xh, Xl, Yh, Yl

template <bool X3>
__device__ __forceinline__ void fwd_gen(const PhaseRec *__restrict__ tab, int64_t n, int64_t chunk, int f0,
                                        char *arr_h, char *arr_l, int gt) {
    const int k = gt >> 3, r = gt & 7;
    const int64_t ib = chunk * FKB + k;
    const bool valid = ib < n;
    const int u0 = f0 + 32 * r;
    Cheb ca, sb;
    float size = 0.0f;
    if (valid) {
        const PhaseRec R = tab[ib];
        float c0, s0, cb0, sb0;
        seed_phasor(u0, R.ta, c0, s0);
        seed_phasor(u0, R.tb, cb0, sb0);
        ca.f = c0;
        ca.fm = c0 * R.ca + s0 * R.sa;            // cos((u0 - 1) alpha)
        ca.ch = R.c2ah; ca.cl = R.c2al;
        sb.f = 2.0f * sb0;                         // 2 sin(u0 beta)
        sb.fm = 2.0f * (sb0 * R.cb - cb0 * R.sb);  // 2 sin((u0 - 1) beta)
        sb.ch = R.c2bh; sb.cl = R.c2bl;
        size = R.size;
    } else {
        ca.f = ca.fm = ca.ch = ca.cl = 0.0f;
        sb.f = sb.fm = sb.ch = sb.cl = 0.0f;
    }
    float v[32];
    v[0] = ca.f * sb.f;
#pragma unroll
    for (int j = 1; j < 32; ++j) v[j] = ca.next() * sb.next();
    if (u0 == 0) v[0] = size;
    unsigned h[16], l[16];
#pragma unroll
    for (int m = 0; m < 16; ++m) {
        if (X3) {
            split2(v[2 * m], v[2 * m + 1], h[m], l[m]);
        } else {
            h[m] = pack_bf16(v[2 * m], v[2 * m + 1]);
        }
    }
    char *ph = arr_h + k * FROW + r * 64;
#pragma unroll
    for (int m = 0; m < 4; ++m)
        *(u32x4 *)(ph + 16 * m) = u32x4{h[4 * m], h[4 * m + 1], h[4 * m + 2], h[4 * m + 3]};
    if (X3) {
        char *pl = arr_l + k * FROW + r * 64;
#pragma unroll
        for (int m = 0; m < 4; ++m)
            *(u32x4 *)(pl + 16 * m) = u32x4{l[4 * m], l[4 * m + 1], l[4 * m + 2], l[4 * m + 3]};
    }
}

// One 32 x 16 MFMA operand (rows f_base..f_base+31 of the frequency axis, blocks kbase..kbase+15)
// from an LDS [block][frequency] array, with two transpose reads.
__device__ __forceinline__ bf16x8 load_opT(const char *arr, int f_base, int kbase, int lane) {
    const int q = lane >> 4, i = lane & 15;
    const int row = kbase + 8 * (q >> 1) + (i >> 2);
    const int col = f_base + 16 * (q & 1) + 4 * (i & 3);
    typedef __attribute__((address_space(3))) s16x4 lds_s16x4;
    const lds_s16x4 *p0 = (const lds_s16x4 *)(arr + row * FROW + col * 2);
    const lds_s16x4 *p1 = (const lds_s16x4 *)(arr + (row + 4) * FROW + col * 2);
    const s16x4 a = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_s16x4 *)p0);
    const s16x4 b = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_s16x4 *)p1);
    typedef short s16x8 __attribute__((ext_vector_type(8)));
    const s16x8 c = {a[0], a[1], a[2], a[3], b[0], b[1], b[2], b[3]};
    return __builtin_bit_cast(bf16x8, c);
}

template <bool X3>
__device__ __forceinline__ void fwd_mma(const char *buf, int wu, int wp, int lane, f32x16 (&acc)[4][2]) {
    const char *xh = buf, *xl = buf + FARR, *yh = buf + 2 * FARR, *yl = buf + 3 * FARR;
#pragma unroll
    for (int ks = 0; ks < FKB / 16; ++ks) {
        bf16x8 ah[4], al[4], bh[2], bl[2];
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            ah[a] = load_opT(xh, wu + 32 * a, 16 * ks, lane);
            if (X3) al[a] = load_opT(xl, wu + 32 * a, 16 * ks, lane);
        }
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            bh[b] = load_opT(yh, wp + 32 * b, 16 * ks, lane);
            if (X3) bl[b] = load_opT(yl, wp + 32 * b, 16 * ks, lane);
        }
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[a], bh[b], acc[a][b], 0, 0, 0);
                if (X3) {
                    acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[a], bl[b], acc[a][b], 0, 0, 0);
                    acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[a], bh[b], acc[a][b], 0, 0, 0);
                }
            }
    }
}

template <bool X3>
__global__ __launch_bounds__(512) void k_fwd_bf16(int64_t n, int Mu, int Mp, const PhaseRec *__restrict__ tx,
                                                  const PhaseRec *__restrict__ ty, float *__restrict__ part,
                                                  int tiles_p, int64_t chunks, int64_t chunks_per_split) {
    __shared__ __attribute__((aligned(16))) char smem[2 * FBUF];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int group = wave >> 2, gt = tid & 255;
    const int tu0 = (int)(blockIdx.x / tiles_p) * FT, tp0 = (int)(blockIdx.x % tiles_p) * FT;
    const int wu = 128 * (wave >> 2), wp = 64 * (wave & 3);
    const int64_t c_begin = (int64_t)blockIdx.y * chunks_per_split;
    const int64_t c_end = min(chunks, c_begin + chunks_per_split);

    f32x16 acc[4][2];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[a][b][r] = 0.0f;

    if (c_begin < c_end) {
        if (group == 0) fwd_gen<X3>(tx, n, c_begin, tu0, smem, smem + FARR, gt);
        else fwd_gen<X3>(ty, n, c_begin, tp0, smem + 2 * FARR, smem + 3 * FARR, gt);
    }
    __syncthreads();
    for (int64_t c = c_begin; c < c_end; ++c) {
        const int bsel = (int)((c - c_begin) & 1);
        char *cur = smem + bsel * FBUF, *nxt = smem + (bsel ^ 1) * FBUF;
        const bool more = c + 1 < c_end;
        if (group == 0) {
            fwd_mma<X3>(cur, wu, wp, lane, acc);
            if (more) fwd_gen<X3>(tx, n, c + 1, tu0, nxt, nxt + FARR, gt);
        } else {
            if (more) fwd_gen<X3>(ty, n, c + 1, tp0, nxt + 2 * FARR, nxt + 3 * FARR, gt);
            fwd_mma<X3>(cur, wu, wp, lane, acc);
        }
        __syncthreads();
    }

    float *out = part + (size_t)blockIdx.y * (size_t)Mu * (size_t)Mp;
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int u = tu0 + wu + 32 * a + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                const int p = tp0 + wp + 32 * b + (lane & 31);
                if (u < Mu && p < Mp) out[(size_t)u * Mp + p] = acc[a][b][r];
            }
}

// ================================================================================================
// Backward: G[i][nn] = sum_k A_ik B[k][nn], g_i = sum_nn E_i,nn G[i][nn].
// 512 threads = 8 waves; wave w owns blocks i0 + 32 w .. + 31 and all 256 columns of the N tile.
// A (sine differences along the K axis) is generated in registers directly in MFMA operand
// layout: the lane half h = lane / 32 walks frequencies h * Kh + 8 t (t = 0, 1, ...), so each
// lane's frequencies are contiguous and its recurrence never restarts except to reseed.
// B is staged per chunk of 16 + 16 frequencies in LDS ([column][32] bf16, rows of 80 bytes).
// Global B is pre-tiled: tile (n_tile, q) is a contiguous [256][32] block, hi and lo separately.
// ================================================================================================
constexpr int BTN = 256;           // N tile (columns)
constexpr int BROW = 80;           // LDS bytes per column row (32 bf16 + pad)
constexpr int BARR = BTN * BROW;   // bytes per hi or lo array
constexpr int BBUF = 2 * BARR;

template <bool X3>
__device__ __forceinline__ void bwd_load_b(const unsigned short *__restrict__ gh, const unsigned short *__restrict__ gl,
                                           char *buf, int tid) {
    // 256 rows x 32 bf16 = 16 KB per array: thread t copies 32 bytes of row t/2.
    const int row = tid >> 1, half = tid & 1;
    const u32x4 *sh = (const u32x4 *)(gh + row * 32 + half * 16);
    const u32x4 v0 = sh[0], v1 = sh[1];
    *(u32x4 *)(buf + row * BROW + half * 32) = v0;
    *(u32x4 *)(buf + row * BROW + half * 32 + 16) = v1;
    if (X3) {
        const u32x4 *sl = (const u32x4 *)(gl + row * 32 + half * 16);
        const u32x4 w0 = sl[0], w1 = sl[1];
        *(u32x4 *)(buf + BARR + row * BROW + half * 32) = w0;
        *(u32x4 *)(buf + BARR + row * BROW + half * 32 + 16) = w1;
    }
}

template <bool X3>
__global__ __launch_bounds__(512) void k_bwd_bf16(int64_t n, BwdAxisBf16 ax) {
    __shared__ __attribute__((aligned(16))) char smem[2 * BBUF];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int h = lane >> 5, j = lane & 31;
    const int64_t i0 = (int64_t)blockIdx.x * 256 + 32 * wave;
    const int ntile = blockIdx.y, n0 = ntile * BTN;
    const int64_t ib = i0 + j;        // this lane's block for the A operand
    const bool valid = ib < n;
    const int Q = ax.Kh / 16;         // chunks along K

    // A-operand recurrence state (basis along the K axis).
    PhaseRec RA;
    if (valid) RA = ax.ta[ib];
    Cheb ca, sb;
    int kcur = h * ax.Kh;             // next frequency this lane generates
    auto reseed = [&]() {
        if (valid) {
            float c0, s0, cb0, sb0;
            seed_phasor(kcur, RA.ta, c0, s0);
            seed_phasor(kcur, RA.tb, cb0, sb0);
            ca.f = c0; ca.fm = c0 * RA.ca + s0 * RA.sa; ca.ch = RA.c2ah; ca.cl = RA.c2al;
            sb.f = 2.0f * sb0; sb.fm = 2.0f * (sb0 * RA.cb - cb0 * RA.sb); sb.ch = RA.c2bh; sb.cl = RA.c2bl;
        } else {
            ca.f = ca.fm = ca.ch = ca.cl = 0.0f;
            sb.f = sb.fm = sb.ch = sb.cl = 0.0f;
        }
    };
    reseed();
    int since = 0;

    f32x16 acc[8];
#pragma unroll
    for (int b = 0; b < 8; ++b)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[b][r] = 0.0f;

    const size_t tile_elems = (size_t)BTN * 32;
    const unsigned short *gbh = ax.Bh + (size_t)ntile * Q * tile_elems;
    const unsigned short *gbl = X3 ? ax.Bl + (size_t)ntile * Q * tile_elems : nullptr;

    bwd_load_b<X3>(gbh, gbl, smem, tid);
    __syncthreads();
    for (int q = 0; q < Q; ++q) {
        char *cur = smem + (q & 1) * BBUF, *nxt = smem + ((q & 1) ^ 1) * BBUF;
        if (q + 1 < Q)
            bwd_load_b<X3>(gbh + (size_t)(q + 1) * tile_elems, X3 ? gbl + (size_t)(q + 1) * tile_elems : nullptr,
                           nxt, tid);
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            // 8 consecutive basis values of this lane's block.
            if (since == 4) { reseed(); since = 0; }
            float v[8];
            v[0] = ca.f * sb.f;
#pragma unroll
            for (int e = 1; e < 8; ++e) v[e] = ca.next() * sb.next();
            ca.next(); sb.next();
            if (kcur == 0) v[0] = valid ? RA.size : 0.0f;
            kcur += 8;
            ++since;
            unsigned hh[4], ll[4];
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                if (X3) split2(v[2 * m], v[2 * m + 1], hh[m], ll[m]);
                else hh[m] = pack_bf16(v[2 * m], v[2 * m + 1]);
            }
            const bf16x8 ah = __builtin_bit_cast(bf16x8, u32x4{hh[0], hh[1], hh[2], hh[3]});
            bf16x8 al;
            if (X3) al = __builtin_bit_cast(bf16x8, u32x4{ll[0], ll[1], ll[2], ll[3]});
#pragma unroll
            for (int b = 0; b < 8; ++b) {
                const int off = (32 * b + j) * BROW + h * 32 + s * 16;
                const bf16x8 bh = *(const bf16x8 *)(cur + off);
                acc[b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bh, acc[b], 0, 0, 0);
                if (X3) {
                    const bf16x8 bl = *(const bf16x8 *)(cur + BARR + off);
                    acc[b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bl, acc[b], 0, 0, 0);
                    acc[b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bh, acc[b], 0, 0, 0);
                }
            }
        }
        __syncthreads();
    }

    // Epilogue: lane holds G for rows 8 (r / 4) + 4 h + r % 4 and columns n0 + 32 b + j.
    // E = -2 sin(nn alpha) sin(nn beta) of the epilogue axis, stepped by 32 columns.
    float rs[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int row = 8 * (r >> 2) + 4 * h + (r & 3);
        const int64_t ibe = i0 + row;
        float sum = 0.0f;
        if (ibe < n) {
            const PhaseRec RE = ax.te[ibe];
            const int nn = n0 + j;
            float ca0, sa0, cb0, sb0;
            seed_phasor(nn, RE.ta, ca0, sa0);
            seed_phasor(nn, RE.tb, cb0, sb0);
#pragma unroll
            for (int b = 0; b < 8; ++b) {
                sum = fmaf(-2.0f * sa0 * sb0, acc[b][r], sum);
                const float ta = ca0 * RE.ca32 - sa0 * RE.sa32;
                sa0 = sa0 * RE.ca32 + ca0 * RE.sa32;
                ca0 = ta;
                const float tb = cb0 * RE.cb32 - sb0 * RE.sb32;
                sb0 = sb0 * RE.cb32 + cb0 * RE.sb32;
                cb0 = tb;
            }
        }
        rs[r] = sum;
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        float v = rs[r];
        v += __shfl_xor(v, 1);
        v += __shfl_xor(v, 2);
        v += __shfl_xor(v, 4);
        v += __shfl_xor(v, 8);
        v += __shfl_xor(v, 16);
        rs[r] = v;
    }
    if (j == 0) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int64_t ibe = i0 + 8 * (r >> 2) + 4 * h + (r & 3);
            if (ibe < n) ax.gpart[(size_t)ntile * (size_t)n + (size_t)ibe] = (double)rs[r];
        }
    }
}

// Backward operand preparation for the bf16 path: BT[nn][k] = a_up / (scale of the K axis),
// split into bf16 hi and lo, zero padded to [Np][2 Kh] and tiled as
// [n_tile][q][row][half * 16 + j] (k = half * Kh + 16 q + j).
// trans = 0: nn = u, k = p (gx operand, a_up / vt_p);  trans = 1: nn = p, k = u (gy, a_up / wt_u).
__global__ void k_prep_bwd_bf16(const double *__restrict__ a, int Mu, int Mp, double W, double H, int trans,
                                int Np, int Kh, unsigned short *__restrict__ Bh, unsigned short *__restrict__ Bl) {
    const size_t total = (size_t)Np * (size_t)(2 * Kh);
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= total) return;
    // decode the tiled position
    const int Q = Kh / 16;
    const size_t tile = idx / (256 * 32);
    const int within = (int)(idx % (256 * 32));
    const int row = within / 32, col = within % 32;
    const int nt = (int)(tile / Q), q = (int)(tile % Q);
    const int nn = nt * 256 + row;
    const int half = col / 16, jj = col % 16;
    const int k = half * Kh + 16 * q + jj;
    float hv = 0.0f, lv = 0.0f;
    const int Nb = trans ? Mp : Mu, Ka = trans ? Mu : Mp;
    if (nn < Nb && k < Ka) {
        const int u = trans ? k : nn, p = trans ? nn : k;
        const double av = a[(size_t)u * Mp + p];
        double sc;
        if (trans) sc = u ? (double)u * kPi / W : 1.0;
        else sc = p ? (double)p * kPi / H : 1.0;
        const double v = av / sc;
        hv = (float)(__bf16)(float)v;
        lv = (float)(__bf16)(float)(v - (double)hv);
    }
    Bh[idx] = __builtin_bit_cast(unsigned short, (__bf16)hv);
    Bl[idx] = __builtin_bit_cast(unsigned short, (__bf16)lv);
}

}  // namespace

hipError_t launch_phase_tables(int64_t n, const double *x, const double *y, const double *w, const double *h,
                               double W, double H, PhaseRec *tx, PhaseRec *ty, hipStream_t s) {
    if (n == 0) return hipSuccess;
    const unsigned g = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(k_phase_table, dim3(g), dim3(256), 0, s, n, x, w, W, tx);
    hipLaunchKernelGGL(k_phase_table, dim3(g), dim3(256), 0, s, n, y, h, H, ty);
    return hipGetLastError();
}

hipError_t launch_fwd_bf16(const FwdPlan &pl, bool x3, int64_t n, int Mu, int Mp, const PhaseRec *tx,
                           const PhaseRec *ty, float *part, hipStream_t s) {
    if (pl.tu != FT || pl.tp != FT || pl.kb != FKB) return hipErrorInvalidValue;
    dim3 grid(pl.tiles_u * pl.tiles_p, pl.splits);
    if (x3)
        hipLaunchKernelGGL(k_fwd_bf16<true>, grid, dim3(512), 0, s, n, Mu, Mp, tx, ty, part, pl.tiles_p, pl.chunks,
                           pl.chunks_per_split);
    else
        hipLaunchKernelGGL(k_fwd_bf16<false>, grid, dim3(512), 0, s, n, Mu, Mp, tx, ty, part, pl.tiles_p,
                           pl.chunks, pl.chunks_per_split);
    return hipGetLastError();
}

hipError_t launch_prep_bwd_bf16(const double *a, int Mu, int Mp, double W, double H, int trans, int Np, int Kh,
                                unsigned short *Bh, unsigned short *Bl, hipStream_t s) {
    const size_t total = (size_t)Np * (size_t)(2 * Kh);
    hipLaunchKernelGGL(k_prep_bwd_bf16, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, a, Mu, Mp, W, H,
                       trans, Np, Kh, Bh, Bl);
    return hipGetLastError();
}

hipError_t launch_bwd_bf16(bool x3, int64_t n, const BwdAxisBf16 &ax, hipStream_t s) {
    dim3 grid((unsigned)((n + 255) / 256), (unsigned)((ax.Nb + BTN - 1) / BTN));
    if (x3) hipLaunchKernelGGL(k_bwd_bf16<true>, grid, dim3(512), 0, s, n, ax);
    else hipLaunchKernelGGL(k_bwd_bf16<false>, grid, dim3(512), 0, s, n, ax);
    return hipGetLastError();
}

}  // namespace pp
