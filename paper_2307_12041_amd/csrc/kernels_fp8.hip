// kernels_fp8.hip -- FP8 operand types PP_FP8 and PP_FP8X3: the basis values and the prepared
// coefficient operand in OCP e4m3 (3 mantissa bits), contracted on v_mfma_scale_f32_32x32x64_f8f6f4
// with FP32 accumulation; x3 splits every operand into e4m3 hi + lo and sums hi*hi + lo*hi + hi*lo.
//
// Scales (E8M0, a power of two per 32 K values of one MFMA row or column; the lanes l and l + 32 of
// a row carry the same code, so one scale covers the row's 64 K values of a chunk):
//   * generated basis values (|S| <= 2, |cos| <= 1) are carried as v * 2^7, scale 2^-7;
//   * the coefficient operand of the gradient contraction takes one scale per column and chunk, the
//     smallest power of two that brings the column's largest magnitude to <= 448 (e4m3 max);
//   * the size entries of the basis (S_0 = w, the u = 0 row and p = 0 column of the coefficient
//     contraction) take the scale of the largest size among the chunk's blocks; in the gradient
//     contraction the k = 0 term (size times the k = 0 row of the operand) is added exactly in the
//     FP32 epilogue instead.
// Every value is brought below 448 before conversion (the conversion does not saturate).
//
// Lane layouts (measured on gfx950): operand lane l holds row (or column) l % 32 and 32 K values in
// its 8 registers; A and B use the same K order, so any consistent assignment of K values to
// (lane half, byte) contracts correctly.  ds_read_b64_tr_b8 (16-lane groups, source lane s reading
// 8 bytes): result lane i, byte e is byte i % 8 of the 8 bytes of source lane 2 e + i / 8.
#include "basis_gen.h"

#include <utility>

namespace pp {

using namespace gen;

namespace {

typedef int i32x8 __attribute__((ext_vector_type(8)));
typedef int i32x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

constexpr int kE8One = 127;          // E8M0 code of 2^0
constexpr int kBasisShift = 7;       // generated basis values carried as v * 2^7
constexpr float kBasisMul = 128.0f;
constexpr int kBasisCode = kE8One - kBasisShift;

// Four floats (|x| < 464) to four e4m3 codes, rounded to nearest even; byte e holds x_e.
__device__ __forceinline__ unsigned pk4(float a, float b, float c, float d) {
    const int w = __builtin_amdgcn_cvt_pk_fp8_f32(a, b, 0, false);
    return (unsigned)__builtin_amdgcn_cvt_pk_fp8_f32(c, d, w, true);
}

// hi = e4m3(x), lo = e4m3(x - hi) for four values (x3 split; the remainders are exact in fp32).
__device__ __forceinline__ void split4(float a, float b, float c, float d, unsigned &hi, unsigned &lo) {
    hi = pk4(a, b, c, d);
    const f32x2 h01 = __builtin_amdgcn_cvt_pk_f32_fp8((int)hi, false);
    const f32x2 h23 = __builtin_amdgcn_cvt_pk_f32_fp8((int)hi, true);
    lo = pk4(a - h01[0], b - h01[1], c - h23[0], d - h23[1]);
}

// A scale code held in a register the compiler cannot see through (a constant scale operand would
// be encoded as a floating-point inline constant).
__device__ __forceinline__ int opaque(int v) {
    asm volatile("" : "+v"(v));
    return v;
}

// E8M0 exponent e (code 127 + e) with m * 2^-e <= 448 for the largest magnitude m >= 0 of a group.
__device__ __forceinline__ int e8_exponent(float m) {
    if (!(m > 0.0f)) return 0;
    int e = (int)ceilf(log2f(m * (1.0f / 448.0f)));
    if (ldexpf(m, -e) > 448.0f) ++e;      // log2f rounding
    if (e < -kE8One) e = -kE8One;
    if (e > kE8One) e = kE8One;
    return e;
}

__device__ __forceinline__ void wait_copies() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }
__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// ================================================================================================
// Gradient contraction: G[i][nn] = sum_k A_ik B[k][nn] (A: the K-axis basis, generated; B: the
// prepared coefficient operand), g_i = sum_nn E_i,nn G[i][nn] (the epilogue kinds of the row forms).
// Prepared operand, one 36 KB tile per (N tile, chunk of 64 K values):
//   bytes [0, 32768): 256 rows (nn) of 128 bytes, [hi K 0..63 | lo K 0..63], K value 32 h + e of the
//     chunk being frequency h Kh + 32 q + e; 16-byte segments XOR-swizzled by (row / 2) % 8;
//   bytes [32768, 33792): the E8M0 code of each row (one dword per row, code in byte 0);
//   the rest padding (the tile is copied in 9 slices of 4 KB).
// The k = 0 entry is left out of the e4m3 operand (its basis value is the block size, which the
// basis scale cannot carry); its exact value, one float per nn, goes to B0[nn] for the epilogue.
// ================================================================================================
constexpr int F8_TN = 256;                       // N tile
constexpr int F8_ROW = 128;                      // bytes per operand row (hi + lo)
constexpr int F8_DATA = F8_TN * F8_ROW;          // 32 KB
constexpr int F8_TILE = 9 * 4096;                // data + scales + padding

__device__ __forceinline__ int f8_seg(int row, int seg) { return (seg ^ ((row >> 1) & 7)) << 4; }

}  // namespace

// One thread per (N tile, chunk, row): the 64 values of its row, their scale, hi and lo codes.
// form / trans / sc as in k_prep_bwd_bf16: trans = 0: nn = u, k = p; trans = 1: nn = p, k = u.
__global__ void k_prep_bwd_fp8(int form, const double *__restrict__ a, int Mu, int Mp, double W, double H,
                               int trans, int Np, int Kh, unsigned char *__restrict__ B, float *__restrict__ B0) {
    const int Q = Kh / 32;
    const int64_t rows_total = (int64_t)(Np / F8_TN) * Q * F8_TN;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= rows_total) return;
    const int row = (int)(idx % F8_TN);
    const int64_t tq = idx / F8_TN;
    const int nt = (int)(tq / Q), q = (int)(tq % Q);
    const int nn = nt * F8_TN + row;
    const int Nb = trans ? Mp : Mu, Ka = trans ? Mu : Mp;
    auto value = [&](int k) -> double {
        if (nn >= Nb || k >= Ka) return 0.0;
        const int u = trans ? k : nn, p = trans ? nn : k;
        const double wt = u ? (double)u * kPi / W : 1.0, vt = p ? (double)p * kPi / H : 1.0;
        double sc = 1.0;
        if (form == ROW_FIELD) sc = trans ? wt : vt;
        else if (form == ROW_POTENTIAL) sc = wt * vt;
        return a[(size_t)u * Mp + p] / sc;
    };
    float v[64];
    float m = 0.0f;
#pragma unroll 8
    for (int c = 0; c < 64; ++c) {
        const int k = (c >> 5) * Kh + 32 * q + (c & 31);
        v[c] = k == 0 ? 0.0f : (float)value(k);
        m = fmaxf(m, fabsf(v[c]));
    }
    const int e = e8_exponent(m);
    unsigned char *tile = B + (size_t)tq * F8_TILE;
    unsigned hi[16], lo[16];
#pragma unroll
    for (int g = 0; g < 16; ++g) {
        split4(ldexpf(v[4 * g], -e), ldexpf(v[4 * g + 1], -e), ldexpf(v[4 * g + 2], -e), ldexpf(v[4 * g + 3], -e),
               hi[g], lo[g]);
    }
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        *(u32x4 *)(tile + row * F8_ROW + f8_seg(row, s)) = u32x4{hi[4 * s], hi[4 * s + 1], hi[4 * s + 2], hi[4 * s + 3]};
        *(u32x4 *)(tile + row * F8_ROW + f8_seg(row, 4 + s)) =
            u32x4{lo[4 * s], lo[4 * s + 1], lo[4 * s + 2], lo[4 * s + 3]};
    }
    ((int *)(tile + F8_DATA))[row] = kE8One + e;
    if (q == 0) B0[nn] = (float)value(0);
}

namespace {

// Basis generator of one lane for one 32-block subtile: frequencies h Kh + 32 q + e of its block,
// carried as v * 2^7, from FP32 phasors that jump by 32 frequencies per chunk (as in the bf16
// gradient contraction).
template <int KA>
struct Gen8 {
    Cheb ca, sb;
    float pac, pas, pbc, pbs, jac, jas, jbc, jbs, sac, sas, sbc, sbs;

    __device__ __forceinline__ void init(const PhaseRec *__restrict__ tab, int64_t ib, bool valid, int k0) {
        if (valid) {
            const PhaseRec RA = tab[ib];
            seed_phasor(k0, RA.ta, pac, pas);
            seed_phasor(k0, RA.tb, pbc, pbs);
            jac = RA.ca32; jas = RA.sa32; jbc = RA.cb32; jbs = RA.sb32;
            sac = RA.ca; sas = RA.sa; sbc = RA.cb; sbs = RA.sb;
            ca.ch = RA.c2ah; ca.cl = RA.c2al; sb.ch = RA.c2bh; sb.cl = RA.c2bl;
        } else {
            pac = pas = pbc = pbs = jac = jas = jbc = jbs = sac = sas = sbc = sbs = 0.0f;
            ca.ch = ca.cl = sb.ch = sb.cl = 0.0f;
        }
        reseed();
    }
    __device__ __forceinline__ void reseed() {
        if constexpr (KA == RUN_COS) {
            ca.f = kBasisMul * pac;
            ca.fm = kBasisMul * (pac * sac + pas * sas);
        } else {
            ca.f = pac;
            ca.fm = pac * sac + pas * sas;                        // cos((k - 1) alpha)
            sb.f = 2.0f * kBasisMul * pbs;                        // 2^8 sin(k beta)
            sb.fm = 2.0f * kBasisMul * (pbs * sbc - pbc * sbs);   // 2^8 sin((k - 1) beta)
        }
    }
    __device__ __forceinline__ void jump() {
        float t = pac * jac - pas * jas;
        pas = pas * jac + pac * jas;
        pac = t;
        t = pbc * jbc - pbs * jbs;
        pbs = pbs * jbc + pbc * jbs;
        pbc = t;
    }
    // Values 8 p .. 8 p + 7 of the current chunk, split into two hi and two lo dwords.
    template <int P>
    __device__ __forceinline__ void piece(unsigned (&hi)[8], unsigned (&lo)[8]) {
        float v[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            if constexpr (KA == RUN_COS) {
                v[e] = (P == 0 && e == 0) ? ca.f : ca.next1();
            } else {
                v[e] = (P == 0 && e == 0) ? ca.f * sb.f : ca.next1() * sb.next1();
            }
        }
        split4(v[0], v[1], v[2], v[3], hi[2 * P], lo[2 * P]);
        split4(v[4], v[5], v[6], v[7], hi[2 * P + 1], lo[2 * P + 1]);
        if constexpr (P == 3) {
            jump();
            reseed();
        }
    }
};

__device__ __forceinline__ i32x8 as_op(const unsigned (&w)[8]) {
    return i32x8{(int)w[0], (int)w[1], (int)w[2], (int)w[3], (int)w[4], (int)w[5], (int)w[6], (int)w[7]};
}

// One operand tile (chunk at byte offset off of the N tile's operand gtile, gbytes long) into dst, as
// buffer loads into LDS: 16 bytes per thread and slice, each wave's 1 KB at the same offset of the
// buffer.  (The global form of the direct copy is booked by the compiler as an LDS access too, which
// makes every later wait for an LDS read a full one while a copy is in flight; the buffer form counts
// as a memory load only.)
__device__ __forceinline__ void copy_tile8(const char *gtile, int gbytes, unsigned off, char *dst, int tid) {
    typedef __attribute__((address_space(3))) void lds_void;
    const __amdgpu_buffer_rsrc_t rsrc = __builtin_amdgcn_make_buffer_rsrc((void *)gtile, (short)0, gbytes, 0x00020000);
    const int wave = tid >> 6;
#pragma unroll
    for (int s = 0; s < F8_TILE / 4096; ++s)
        __builtin_amdgcn_raw_ptr_buffer_load_lds(rsrc, (lds_void *)(dst + s * 4096 + wave * 1024), 16,
                                                  (unsigned)tid * 16u, off + (unsigned)(s * 4096), 0, 0);
}

// B operand of column tile b from a chunk buffer: lane (j, h) holds row 32 b + j, K values
// 32 h .. 32 h + 31 (hi at logical segments 2 h, 2 h + 1; lo at 4 + 2 h, 5 + 2 h).
__device__ __forceinline__ i32x8 read_b8(const char *buf, int lohi, int b, int h, int j) {
    const int row = 32 * b + j;
    const char *r = buf + row * F8_ROW;
    const u32x4 x = *(const u32x4 *)(r + f8_seg(row, 4 * lohi + 2 * h));
    const u32x4 y = *(const u32x4 *)(r + f8_seg(row, 4 * lohi + 2 * h + 1));
    return i32x8{(int)x[0], (int)x[1], (int)x[2], (int)x[3], (int)y[0], (int)y[1], (int)y[2], (int)y[3]};
}

// 256 threads = 4 waves; wave w owns blocks i0 + 64 w .. + 63 (two 32-block subtiles) and all 256
// columns of the N tile (16 accumulator tiles).  Per chunk of 64 K values: each column tile's B
// operands are read from LDS and contracted with both subtiles' A operands (1 or 3 MFMAs each);
// meanwhile the next chunk's A operands are generated in registers, one eighth per column tile.
// The chunk after next is copied into the buffer released at the chunk's barrier.
template <bool X3, int KA, int E1, int E2>
__global__ __launch_bounds__(256) void k_bwd_fp8(int64_t n, BwdAxisFp8 ax) {
    __shared__ __attribute__((aligned(16))) char smem[2 * F8_TILE];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int h = lane >> 5, j = lane & 31;
    const int btile = blockIdx.x, ntile = blockIdx.y;
    const int64_t i0 = (int64_t)btile * 256 + 64 * wave;
    const int n0 = ntile * F8_TN;
    const int Q = ax.Kh / 32;
    const char *gb = (const char *)ax.B + (size_t)ntile * Q * F8_TILE;

    Gen8<KA> g[2];
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        const int64_t ib = i0 + 32 * a + j;
        g[a].init(ax.ta, ib, ib < n, h * ax.Kh);
    }
    f32x16 acc[2][8];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 8; ++b)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[a][b][r] = 0.0f;

    // chunk 0's A operands and B tile; chunk 1's B tile
    unsigned ah[2][8], al[2][8], nh[2][8], nl[2][8];
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        g[a].template piece<0>(ah[a], al[a]);
        g[a].template piece<1>(ah[a], al[a]);
        g[a].template piece<2>(ah[a], al[a]);
        g[a].template piece<3>(ah[a], al[a]);
    }
    copy_tile8(gb, Q * F8_TILE, 0u, smem, tid);
    if (Q > 1) copy_tile8(gb, Q * F8_TILE, (unsigned)F8_TILE, smem + F8_TILE, tid);
    const int sa = opaque(kBasisCode);
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();

    for (int q = 0; q < Q; ++q) {
        const char *cur = smem + (q & 1) * F8_TILE;
        const int *scl = (const int *)(cur + F8_DATA);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const i32x8 bh = read_b8(cur, 0, b, h, j);
            const i32x8 bl = X3 ? read_b8(cur, 1, b, h, j) : bh;
            const int sb = scl[32 * b + j];
#pragma unroll
            for (int a = 0; a < 2; ++a)
                acc[a][b] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(as_op(ah[a]), bh, acc[a][b], 0, 0, 0, sa,
                                                                             0, sb);
            if constexpr (X3) {
#pragma unroll
                for (int a = 0; a < 2; ++a)
                    acc[a][b] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(as_op(al[a]), bh, acc[a][b], 0, 0, 0,
                                                                                 sa, 0, sb);
#pragma unroll
                for (int a = 0; a < 2; ++a)
                    acc[a][b] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(as_op(ah[a]), bl, acc[a][b], 0, 0, 0,
                                                                                 sa, 0, sb);
            }
            // generator: subtile b / 4, piece b % 4 of the next chunk (past the last chunk the values
            // are generated and never used)
            if (b < 4) {
                if (b == 0) g[0].template piece<0>(nh[0], nl[0]);
                if (b == 1) g[0].template piece<1>(nh[0], nl[0]);
                if (b == 2) g[0].template piece<2>(nh[0], nl[0]);
                if (b == 3) g[0].template piece<3>(nh[0], nl[0]);
            } else {
                if (b == 4) g[1].template piece<0>(nh[1], nl[1]);
                if (b == 5) g[1].template piece<1>(nh[1], nl[1]);
                if (b == 6) g[1].template piece<2>(nh[1], nl[1]);
                if (b == 7) g[1].template piece<3>(nh[1], nl[1]);
            }
        }
        // all reads of this chunk's buffer are done, the next chunk's tile has landed
        wait_copies();
        lds_barrier();
        if (q + 2 < Q) copy_tile8(gb, Q * F8_TILE, (unsigned)(q + 2) * (unsigned)F8_TILE, smem + (q & 1) * F8_TILE, tid);
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int w = 0; w < 8; ++w) {
                ah[a][w] = nh[a][w];
                al[a][w] = nl[a][w];
            }
    }
    wait_copies();
    __syncthreads();

    // Epilogue (as in the bf16 gradient contraction): one column tile at a time transposed through
    // LDS so that lane l holds row l, plus the exact k = 0 term size_i * B0[nn]; each 32-column run
    // summed in FP32, the runs in FP64.
    constexpr int EPS = 36;
    float *tb = (float *)smem + wave * (64 * EPS);
    const int64_t ibr = i0 + lane;
    const bool rvalid = ibr < n;
    EGen<E1, E2> eg;
    const PhaseRec RE = rvalid ? ax.te[ibr] : PhaseRec{};
    eg.init(RE, n0, ax.pil);
    const float size_k = (rvalid && KA == RUN_SINDIFF) ? ax.ta[ibr].size : 0.0f;   // A_i0 of the K axis
    const float *b0 = ax.B0 + n0;
    double sum = 0.0, sum2 = 0.0;
    float g00 = 0.0f;
#pragma unroll
    for (int b = 0; b < 8; ++b) {
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int r = 0; r < 16; ++r) tb[(32 * a + 8 * (r >> 2) + 4 * h + (r & 3)) * EPS + j] = acc[a][b][r];
        float gv[32];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const float4 x = *(const float4 *)(tb + lane * EPS + 4 * k);
            gv[4 * k] = x.x; gv[4 * k + 1] = x.y; gv[4 * k + 2] = x.z; gv[4 * k + 3] = x.w;
        }
        if constexpr (KA == RUN_SINDIFF) {
#pragma unroll
            for (int k = 0; k < 32; ++k) gv[k] = fmaf(size_k, b0[32 * b + k], gv[k]);
        }
        if (b == 0) g00 = gv[0];
        eg.seed();
        float nnp = (float)(n0 + 32 * b) * eg.pil;
        float run = 0.0f, run2 = 0.0f;
#pragma unroll
        for (int k = 0; k < 32; ++k) {
            if constexpr (E1 == RUN_COSDIFF || E1 == RUN_SINDIFF) {
                run = fmaf(eg.c0.f * eg.c1.f, gv[k], run);
            } else if constexpr (E1 == RUN_COS) {
                run = fmaf(eg.c0.f, gv[k], run);
            } else {
                run = fmaf(nnp * eg.c0.f, gv[k], run);
            }
            if constexpr (EGen<E1, E2>::DUAL) run2 = fmaf(nnp * eg.c1.f, gv[k], run2);
            if constexpr (E1 == RUN_WSIN || EGen<E1, E2>::DUAL) nnp += eg.pil;
            eg.c0.next();
            if constexpr (EGen<E1, E2>::HAS_C1) eg.c1.next();
        }
        sum += (double)run;
        if constexpr (EGen<E1, E2>::DUAL) sum2 += (double)run2;
        eg.rotate();
    }
    if constexpr (E1 == RUN_COSDIFF) sum *= -2.0;
    if constexpr (E1 == RUN_SINDIFF) {
        sum *= 2.0;
        if (n0 == 0) sum += (double)eg.size * (double)g00;
    }
    if (rvalid) {
        ax.gpart[(size_t)ntile * (size_t)n + (size_t)ibr] = sum;
        if constexpr (EGen<E1, E2>::DUAL) ax.gpart2[(size_t)ntile * (size_t)n + (size_t)ibr] = sum2;
    }
}

}  // namespace
}  // namespace pp

namespace pp {
namespace {

// ================================================================================================
// Coefficient contraction: At[u][p] = sum_i S_iu T_ip over a range of blocks.  256 threads = 4 waves;
// wave w owns the 128 x 128 sub-tile (u-half w / 2, p-half w % 2) of a 256 x 256 output tile in 16
// accumulator tiles.  Chunks of 64 blocks: while chunk c is contracted from one LDS buffer, every
// thread generates four runs of 32 frequencies of chunk c + 1 (block k = tid % 64, X and Y runs
// tid / 64 and tid / 64 + 4 of the tile) into the other.
// LDS buffer: X hi, X lo, Y hi, Y lo, each [64 blocks][256 frequencies] e4m3, 16-byte segments
// XOR-swizzled by M(row) (g8_swz), then the E8M0 codes of the u = 0 row and the p = 0 column (the
// chunk's largest size).  Operands are read with ds_read_b64_tr_b8: for read t of an
// operand, source lane s of a 16-lane group reads 8 frequencies (16 g + 8 (s % 2) + ..) of block
// row 32 h + 8 t + s / 2, so that result lane i of group g holds frequency 16 g + i of blocks
// 32 h + 8 t .. + 7 (A and B read alike, hence the same K order).
// ================================================================================================
constexpr int G8_ARR = 64 * 256;
constexpr int G8_CODES = 4 * G8_ARR;
constexpr int G8_BUF = 4 * G8_ARR + 256;

// Rows are 256 bytes, one period of the 64 banks, so a 16-byte segment's banks are fixed by its
// index; the LDS serves 128 bytes per pass for these accesses, where the index mod 8 counts.  A
// b128 store pass (8 lanes) writes one segment of 8 aligned rows, and a 16-lane group of a
// transpose read takes one segment of 8 aligned rows, the 32-lane half that segment and the next
// (an even index and its successor).  M(row) = r ^ 8 (r % 2) ^ (row / 8) % 2, r = row % 8, is
// distinct mod 8 over 8 aligned rows and never equals another row's M ^ 1 (so the two segments of a
// read half fill 16 bank groups); its last term makes all 16 rows of an aligned group distinct, for
// stores served 16 lanes (256 bytes) at a time.  (The previous M, 2 r + (row / 8) % 2, took only
// four values mod 8: two-way conflicts, 85 % of the forward's LDS cycles by the bank-conflict counter.)
__device__ __forceinline__ int g8_swz(int row) {
    const int r = row & 7;
    return r ^ ((r & 1) << 3) ^ ((row >> 3) & 1);
}

// One run's start values and the block's recurrence coefficients and size.
struct Rec8 {
    float4 s;   // cf, cfm, sf, sfm
    float4 c;   // c2ah, c2al, c2bh, c2bl
    float size;
};

__device__ __forceinline__ Rec8 load_rec8(const PhaseRec *__restrict__ tab, const RunSeed *__restrict__ seeds,
                                          int64_t rows, int run, int64_t ib) {
    ib = ib < rows ? ib : rows - 1;   // rows past the table: its last row, a zero record
    Rec8 r;
    r.s = *(const float4 *)&seeds[(size_t)run * (size_t)rows + (size_t)ib];
    r.c = *(const float4 *)&tab[ib].c2ah;
    r.size = tab[ib].size;
    return r;
}

__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = fmaxf(v, __shfl_xor(v, off));
    return v;
}

// One run of 32 frequencies of block row k into an array pair: values v * 2^7 (the size entry of
// the u = 0 run carried as size * 2^-e0 instead), split into hi and lo, two 16-byte segments each.
template <bool X3>
__device__ __forceinline__ void gen_run8(const Rec8 &R, bool first, int e0, char *arr_h, char *arr_l, int k,
                                         int rl) {
    Cheb C, S;
    C.f = R.s.x; C.fm = R.s.y; C.ch = R.c.x; C.cl = R.c.y;
    S.f = kBasisMul * R.s.z; S.fm = kBasisMul * R.s.w; S.ch = R.c.z; S.cl = R.c.w;
    float v[32];
    v[0] = first ? ldexpf(R.size, -e0) : C.f * S.f;
#pragma unroll
    for (int e = 1; e < 32; ++e) v[e] = C.next1() * S.next1();
    unsigned hi[8], lo[8];
#pragma unroll
    for (int g = 0; g < 8; ++g) {
        if constexpr (X3) split4(v[4 * g], v[4 * g + 1], v[4 * g + 2], v[4 * g + 3], hi[g], lo[g]);
        else hi[g] = pk4(v[4 * g], v[4 * g + 1], v[4 * g + 2], v[4 * g + 3]);
    }
    const int sw = g8_swz(k);
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        const int off = k * 256 + (((2 * rl + t) ^ sw) << 4);
        *(u32x4 *)(arr_h + off) = u32x4{hi[4 * t], hi[4 * t + 1], hi[4 * t + 2], hi[4 * t + 3]};
        if constexpr (X3) *(u32x4 *)(arr_l + off) = u32x4{lo[4 * t], lo[4 * t + 1], lo[4 * t + 2], lo[4 * t + 3]};
    }
}

// One 32 x 64 operand (32 frequencies from f_base, the chunk's 64 blocks) by four transpose reads.
__device__ __forceinline__ i32x8 read_op8(const char *arr, int f_base, int lane) {
    typedef __attribute__((address_space(3))) i32x2 lds_i32x2;
    const int s = lane & 15, g = (lane >> 4) & 1, h = lane >> 5;
    const int r = s >> 1;   // row 32 h + 8 t + r: g8_swz of it is r ^ 8 (r % 2) ^ (t % 2)
    const int seg = ((f_base >> 4) + g) ^ r ^ ((r & 1) << 3);
    const int base = (32 * h + r) * 256 + 8 * (s & 1);
    i32x8 o;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int off = base + 8 * t * 256 + ((seg ^ (t & 1)) << 4);
        const i32x2 x = __builtin_amdgcn_ds_read_tr8_b64_v2i32((lds_i32x2 *)(arr + off));
        o[2 * t] = x[0];
        o[2 * t + 1] = x[1];
    }
    return o;
}

template <bool X3>
__global__ __launch_bounds__(256) void k_fwd_fp8(int64_t n, int Mu, int Mp, const PhaseRec *__restrict__ tx,
                                                 const PhaseRec *__restrict__ ty, const RunSeed *__restrict__ sx,
                                                 const RunSeed *__restrict__ sy, float *__restrict__ part,
                                                 int tiles_p, int64_t chunks, int64_t chunks_per_split) {
    __shared__ __attribute__((aligned(16))) char smem[2 * G8_BUF];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int64_t rows = phase_rows(n);
    int tile;
    int64_t split;
    fwd_tile_split(tile, split);
    const int tu0 = (tile / tiles_p) * 256, tp0 = (tile % tiles_p) * 256;
    const int wu = 128 * (wave >> 1), wp = 128 * (wave & 1);
    const int64_t c_begin = split * chunks_per_split;
    const int64_t c_end = min(chunks, c_begin + chunks_per_split);

    f32x16 acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[a][b][r] = 0.0f;

    // generator roles: block k of each chunk, runs r and r + 4 of the tile on both axes
    const int k = tid & 63, r = tid >> 6;
    const bool zx = tu0 == 0 && wave == 0, zy = tp0 == 0 && wave == 0;   // wave 0 holds the u = 0 / p = 0 runs
    auto rec = [&](int which, int64_t chunk) {
        const bool y = which >= 2;
        const int rl = r + 4 * (which & 1);
        return load_rec8(y ? ty : tx, y ? sy : sx, rows, (y ? tp0 : tu0) / 32 + rl, chunk * 64 + k);
    };
    auto gen = [&](int which, const Rec8 &R, char *buf) {
        const bool y = which >= 2;
        const int rl = r + 4 * (which & 1);
        const bool first = (which & 1) == 0 && (y ? zy : zx);   // the run that holds the size entry
        int e0 = 0;
        if (first) {
            e0 = e8_exponent(wave_max(R.size));
            if (lane == 0) ((int *)(buf + G8_CODES))[y ? 1 : 0] = kE8One + e0;
        }
        gen_run8<X3>(R, first, e0, buf + (y ? 2 : 0) * G8_ARR, buf + (y ? 3 : 1) * G8_ARR, k, rl);
    };

    // scales of this wave's operand rows / columns: the u = 0 row (lanes 0 and 32 of subtile 0 of the
    // waves at wu = 0 of the first u tile) and the p = 0 column take the chunk's size code
    const bool lx0 = tu0 + wu == 0 && (lane & 31) == 0;
    const bool ly0 = tp0 + wp == 0 && (lane & 31) == 0;
    const int sbase = opaque(kBasisCode);

    Rec8 R[4];
    if (c_begin < c_end) {
#pragma unroll
        for (int w = 0; w < 4; ++w) gen(w, rec(w, c_begin), smem);
#pragma unroll
        for (int w = 0; w < 4; ++w) R[w] = rec(w, c_begin + 1);
    }
    lds_barrier();
    for (int64_t c = c_begin; c < c_end; ++c) {
        const int bsel = (int)((c - c_begin) & 1);
        char *cur = smem + bsel * G8_BUF, *nxt = smem + (bsel ^ 1) * G8_BUF;
        const int *codes = (const int *)(cur + G8_CODES);
        const int cx = lx0 ? codes[0] : sbase, cy = ly0 ? codes[1] : sbase;
        i32x8 ah[4], al[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            ah[a] = read_op8(cur, wu + 32 * a, lane);
            if constexpr (X3) al[a] = read_op8(cur + G8_ARR, wu + 32 * a, lane);
        }
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const i32x8 bh = read_op8(cur + 2 * G8_ARR, wp + 32 * b, lane);
            const i32x8 bl = X3 ? read_op8(cur + 3 * G8_ARR, wp + 32 * b, lane) : bh;
            const int sb = b == 0 ? cy : sbase;
#pragma unroll
            for (int a = 0; a < 4; ++a) {
                const int sa = a == 0 ? cx : sbase;
                acc[a][b] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(ah[a], bh, acc[a][b], 0, 0, 0, sa, 0, sb);
            }
            if constexpr (X3) {
#pragma unroll
                for (int a = 0; a < 4; ++a) {
                    const int sa = a == 0 ? cx : sbase;
                    acc[a][b] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(al[a], bh, acc[a][b], 0, 0, 0, sa, 0,
                                                                                 sb);
                }
#pragma unroll
                for (int a = 0; a < 4; ++a) {
                    const int sa = a == 0 ? cx : sbase;
                    acc[a][b] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(ah[a], bl, acc[a][b], 0, 0, 0, sa, 0,
                                                                                 sb);
                }
            }
            // run b of the next chunk (past the range: zero or next-split records into the idle buffer)
            gen(b, R[b], nxt);
            R[b] = rec(b, c + 2);
        }
        lds_barrier();
    }

    float *out = part + (size_t)split * (size_t)Mu * (size_t)Mp;
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                const int u = tu0 + wu + 32 * a + 8 * (e >> 2) + 4 * (lane >> 5) + (e & 3);
                const int p = tp0 + wp + 32 * b + (lane & 31);
                if (u < Mu && p < Mp) out[(size_t)u * Mp + p] = acc[a][b][e];
            }
}

}  // namespace

hipError_t launch_fwd_fp8(const FwdPlan &pl, bool x3, int64_t n, int Mu, int Mp, const PhaseRec *tx,
                          const PhaseRec *ty, const RunSeed *sx, const RunSeed *sy, float *part, hipStream_t s) {
    if (pl.tu != 256 || pl.tp != 256 || pl.kb != 64) return hipErrorInvalidValue;
    dim3 grid(pl.tiles_u * pl.tiles_p, pl.splits);
    if (x3)
        hipLaunchKernelGGL(k_fwd_fp8<true>, grid, dim3(256), 0, s, n, Mu, Mp, tx, ty, sx, sy, part, pl.tiles_p,
                           pl.chunks, pl.chunks_per_split);
    else
        hipLaunchKernelGGL(k_fwd_fp8<false>, grid, dim3(256), 0, s, n, Mu, Mp, tx, ty, sx, sy, part, pl.tiles_p,
                           pl.chunks, pl.chunks_per_split);
    return hipGetLastError();
}

size_t fp8_operand_bytes(int Np, int Kh) { return (size_t)(Np / F8_TN) * (size_t)(Kh / 32) * (size_t)F8_TILE; }

hipError_t launch_prep_bwd_fp8(RowForm f, const double *a, int Mu, int Mp, double W, double H, int trans, int Np,
                               int Kh, unsigned char *B, float *B0, hipStream_t s) {
    const int64_t rows = (int64_t)(Np / F8_TN) * (Kh / 32) * F8_TN;
    if (rows == 0) return hipSuccess;
    hipLaunchKernelGGL(k_prep_bwd_fp8, dim3((unsigned)((rows + 255) / 256)), dim3(256), 0, s, (int)f, a, Mu, Mp, W, H,
                       trans, Np, Kh, B, B0);
    return hipGetLastError();
}

hipError_t launch_bwd_fp8(RowForm f, bool x3, int64_t n, const BwdAxisFp8 &ax, hipStream_t s) {
    if (n == 0) return hipSuccess;
    if (f != ROW_FIELD) return hipErrorInvalidValue;
    dim3 grid((unsigned)((n + 255) / 256), (unsigned)((ax.Nb + F8_TN - 1) / F8_TN));
    if (x3) hipLaunchKernelGGL((k_bwd_fp8<true, RUN_SINDIFF, RUN_COSDIFF, -1>), grid, dim3(256), 0, s, n, ax);
    else hipLaunchKernelGGL((k_bwd_fp8<false, RUN_SINDIFF, RUN_COSDIFF, -1>), grid, dim3(256), 0, s, n, ax);
    return hipGetLastError();
}

}  // namespace pp
