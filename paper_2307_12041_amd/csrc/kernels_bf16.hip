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
#include "basis_gen.h"

#include <utility>

namespace pp {

using namespace gen;

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef short s16x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned u32x2 __attribute__((ext_vector_type(2)));


__device__ __forceinline__ unsigned pack_bf16(float a, float b) {
    bf16x2 v = {(__bf16)a, (__bf16)b};
    return __builtin_bit_cast(unsigned, v);
}

// The lo half of a split: packed bf16 of a - ha and b - hb, where ha, hb are the hi parts as fp32
// bit patterns.  Contraction is off so that the remainders are taken from the rounded fp32 values
// wherever a generator splits (a product fused into the subtraction would give other bits than a
// generator whose product is kept for the hi half, and stored and regenerated tables must agree).
__device__ __forceinline__ unsigned split_lo(float a, float b, unsigned ha, unsigned hb) {
#pragma clang fp contract(off)
    return pack_bf16(a - __builtin_bit_cast(float, ha), b - __builtin_bit_cast(float, hb));
}

// Split two fp32 values into packed bf16 hi (round to nearest even) and packed bf16 lo of the
// remainders (exact in fp32).  Plain VALU shifts and subtractions: a bf16 dot-product form of the
// remainder issues fewer instructions but shares the matrix pipe and stalls behind the MFMAs that
// the other wave of the SIMD runs meanwhile (measured 4.8x slower there, against 1.6x for this).
__device__ __forceinline__ void split2(float a, float b, unsigned &hi, unsigned &lo) {
    hi = pack_bf16(a, b);
    lo = split_lo(a, b, hi << 16, hi & 0xffff0000u);
}


}  // namespace

// Per-block phase record for one axis (see common.h); rows n .. rows - 1 get zero records.
__global__ void k_phase_table(int64_t n, int64_t rows, const double *__restrict__ c, const double *__restrict__ sz,
                              double L, PhaseRec *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= rows) return;
    if (i >= n) {
        out[i] = PhaseRec{};
        return;
    }
    const double szi = sz ? sz[i] : 0.0;
    const double ta = c[i] / L, tb = szi / (2.0 * L);
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
    r.size = (float)szi;
    r.pad0 = r.pad1 = r.pad2 = 0.0f;
    out[i] = r;
}

// Run seeds of one axis (see RunSeed in common.h): one thread per row walks the runs, rotating the
// FP64 phasors of u0 alpha and u0 beta by 32 frequencies per run and reseeding them exactly (FP64
// reduction and sincospi) every 16 runs; rows n .. rows - 1 get zero seeds (an absent block).
__global__ void k_seed_table(int64_t n, int64_t rows, int runs, const PhaseRec *__restrict__ tab,
                             RunSeed *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= rows) return;
    if (i >= n) {
        for (int r = 0; r < runs; ++r) out[(size_t)r * (size_t)rows + (size_t)i] = RunSeed{0.0f, 0.0f, 0.0f, 0.0f};
        return;
    }
    const double ta = tab[i].ta, tb = tab[i].tb;
    double sa1, ca1, sb1, cb1, sj, cj, sjb, cjb;
    sincospi(reduce_half_turns(ta), &sa1, &ca1);
    sincospi(reduce_half_turns(tb), &sb1, &cb1);
    sincospi(reduce_half_turns(32.0 * ta), &sj, &cj);
    sincospi(reduce_half_turns(32.0 * tb), &sjb, &cjb);
    double ca = 1.0, sa = 0.0, cb = 1.0, sb = 0.0;   // phasors of u0 alpha and u0 beta
    for (int r = 0; r < runs; ++r) {
        if ((r & 15) == 0) {
            sincospi(reduce_half_turns((double)(32 * r) * ta), &sa, &ca);
            sincospi(reduce_half_turns((double)(32 * r) * tb), &sb, &cb);
        }
        RunSeed q;
        q.cf = (float)ca;
        q.cfm = (float)(ca * ca1 + sa * sa1);           // cos((u0 - 1) alpha)
        q.sf = (float)(2.0 * sb);
        q.sfm = (float)(2.0 * (sb * cb1 - cb * sb1));   // 2 sin((u0 - 1) beta)
        out[(size_t)r * (size_t)rows + (size_t)i] = q;
        const double ta2 = ca * cj - sa * sj, tb2 = cb * cjb - sb * sjb;
        sa = sa * cj + ca * sj;
        ca = ta2;
        sb = sb * cjb + cb * sjb;
        cb = tb2;
    }
}

namespace {

__device__ __forceinline__ void wait_copies() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

// Workgroup barrier that orders LDS only: this wave's LDS operations complete, then all waves meet.
// (__syncthreads() also waits for every outstanding global load, which would expose the latency of
// the record fetches and tile copies that are meant to stay in flight across a phase boundary; the
// tile copies are waited for explicitly before the barrier that hands their buffer over.)
__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// ================================================================================================
// Forward: At[u][p] = sum_i S_iu T_ip over a range of blocks.
// Kernels: k_fwd1_bf16<X3> (one wave per SIMD, three products or one, further below) and the
// store-mode k_fwd_bf16_st (512 threads = 8 waves, wave w owning the 128 x 64 output sub-tile (u-half
// w / 4, p-quarter w % 4), contracting tiles staged from the stored tables with fwd_mma).
// LDS tile layout: [block][frequency] bf16, 512-byte rows with XOR-swizzled 16-byte segments;
// MFMA operands are read with the transpose read.
// ================================================================================================
constexpr int FT = 256;              // output tile (u and p)
constexpr int FKB = 32;              // blocks per chunk
constexpr int FROW = FT * 2;         // bytes per LDS row
constexpr int FARR = FKB * FROW;     // bytes per array
constexpr int FBUF = 4 * FARR;       // Xh, Xl, Yh, Yl

// Byte offset of 16-byte segment `seg` of row `k` in an LDS tile.  The LDS has 64 banks of 4 bytes
// (a 256-byte period, half a row), so a segment's bank group is its index mod 16 for reads; the b128
// stores are served 8 lanes (128 bytes) at a time, where the index mod 8 counts.  The index is
// XORed with M(k) = 4 (k % 4) + (k / 4) % 4, with bit 1 also flipped by bit 1 of k:
//   * a b128 store by 8 (or 16) lanes writes one segment of 8 (or 16) consecutive rows (see fwd_gen);
//     M mod 8 differs across any 8 consecutive aligned rows and M is a bijection on k % 16, so the
//     stores hit distinct bank groups;
//   * a 32-lane half of a transpose read covers 4 consecutive rows k0 .. k0 + 3 (k0 % 4 = 0) and 4
//     consecutive segments of an aligned group of 4; M(k) / 4 = k % 4 moves each row's 4 segments
//     to a different aligned group, so the 16 segments hit 16 distinct bank groups.
// (Measured with the LDS bank-conflict counter: no conflicts for either pattern.)
__device__ __forceinline__ int fswz_mask(int k) {
    return (((k & 3) << 2) | ((k >> 2) & 3)) ^ (((k >> 1) & 1) << 1);
}
__device__ __forceinline__ int fswz(int k, int seg) { return k * FROW + ((seg ^ fswz_mask(k)) << 4); }

// What a generating thread needs for one run of 32 frequencies of one block, held in registers so
// that it can be fetched one phase ahead of its use: the run's seeds (RunSeed) and the block's
// recurrence coefficients and size.
struct GenRec {
    RunSeed s;
    float c2ah, c2al, c2bh, c2bl, size;
};

__device__ __forceinline__ GenRec gen_rec_zero() {
    GenRec g;
    g.s = RunSeed{0.0f, 0.0f, 0.0f, 0.0f};
    g.c2ah = g.c2al = g.c2bh = g.c2bl = g.size = 0.0f;
    return g;
}

// Run `run` of table row ib (the rows are padded: a row past n holds zero seeds, an absent block).
__device__ __forceinline__ GenRec load_gen(const PhaseRec *__restrict__ tab, const RunSeed *__restrict__ seeds,
                                           int64_t rows, int run, int64_t ib) {
    GenRec g;
    g.s = seeds[(size_t)run * (size_t)rows + (size_t)ib];
    const float4 c = *(const float4 *)&tab[ib].c2ah;
    g.c2ah = c.x; g.c2al = c.y; g.c2bh = c.z; g.c2bl = c.w;
    g.size = tab[ib].size;
    return g;
}

// The same with a bounds test (ib >= n gives an absent block).
__device__ __forceinline__ GenRec load_gen_at(const PhaseRec *__restrict__ tab, const RunSeed *__restrict__ seeds,
                                              int64_t rows, int run, int64_t n, int64_t ib) {
    return ib < n ? load_gen(tab, seeds, rows, run, ib) : gen_rec_zero();
}

// Start both recurrences of a run (cos(u alpha) and 2 sin(u beta) at u0 and u0 - 1).
__device__ __forceinline__ void start_run(const GenRec &R, Cheb &ca, Cheb &sb) {
    ca.f = R.s.cf; ca.fm = R.s.cfm; ca.ch = R.c2ah; ca.cl = R.c2al;
    sb.f = R.s.sf; sb.fm = R.s.sfm; sb.ch = R.c2bh; sb.cl = R.c2bl;
}

// The basis values S_u (u0 <= u < u0 + 32) of one run (S_0 = size); the same arithmetic as the
// generating forwards (fwd_gen, RunStages), so stored and regenerated tables agree bit for bit.
__device__ __forceinline__ void gen32(const GenRec &R, int u0, float (&v)[32]) {
    Cheb ca, sb;
    start_run(R, ca, sb);
    v[0] = ca.f * sb.f;
#pragma unroll
    for (int j = 1; j < 32; ++j) v[j] = ca.next1() * sb.next1();
    if (u0 == 0) v[0] = R.size;
}

// 32 consecutive frequencies f0 + 32 r .. + 31 of block k of the chunk, split hi/lo and stored.
// Thread gt of the generating group handles block k = gt % 32 and run r = gt / 32 (R: that run's
// seeds), so the 16 lanes of each store share the segment and cover 16 consecutive rows.
template <bool X3>
__device__ __forceinline__ void fwd_gen(const GenRec &R, int f0, char *arr_h, char *arr_l, int gt) {
    const int k = gt & 31, r = gt >> 5;
    float v[32];
    gen32(R, f0 + 32 * r, v);
    // Split and store one 16-byte segment (8 frequencies) at a time.
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        unsigned h[4], l[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            if (X3) split2(v[8 * m + 2 * e], v[8 * m + 2 * e + 1], h[e], l[e]);
            else h[e] = pack_bf16(v[8 * m + 2 * e], v[8 * m + 2 * e + 1]);
        }
        *(u32x4 *)(arr_h + fswz(k, 4 * r + m)) = u32x4{h[0], h[1], h[2], h[3]};
        if (X3) *(u32x4 *)(arr_l + fswz(k, 4 * r + m)) = u32x4{l[0], l[1], l[2], l[3]};
    }
}

// Lane-dependent byte offsets for the transpose reads of one wave's operands.  An operand covers
// frequencies f_base + 32 a .. + 31 (a = subtile) and blocks 16 ks .. + 15; lane (q = lane / 16,
// i = lane % 16) reads 8 bytes at row r = 8 (q / 2) + i / 4 + 4 rd (rd = read half, + 16 ks) and
// frequency f = f_base + 32 a + 16 (q % 2) + 4 (i % 4).  M(r + 16) = M(r), so one base per
// (subtile, read half) serves both K steps (+ 8192 bytes).
struct OpBase {
    int b[4][2];   // [subtile][read half]
    __device__ __forceinline__ void init(int f_base, int lane) {
        const int q = lane >> 4, i = lane & 15;
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int rd = 0; rd < 2; ++rd) {
                const int row = 8 * (q >> 1) + (i >> 2) + 4 * rd;
                const int col = f_base + 32 * a + 16 * (q & 1) + 4 * (i & 3);
                b[a][rd] = fswz(row, col >> 3) + (col & 7) * 2;
            }
    }
};

// One 32 x 16 MFMA operand from an LDS [block][frequency] array: two transpose reads.
__device__ __forceinline__ bf16x8 load_opT(const char *arr, const OpBase &ob, int a, int ks) {
    typedef __attribute__((address_space(3))) s16x4 lds_s16x4;
    const int off = 8192 * ks;
    const s16x4 x = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_s16x4 *)(arr + ob.b[a][0] + off));
    const s16x4 y = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_s16x4 *)(arr + ob.b[a][1] + off));
    typedef short s16x8 __attribute__((ext_vector_type(8)));
    const s16x8 c = {x[0], x[1], x[2], x[3], y[0], y[1], y[2], y[3]};
    return __builtin_bit_cast(bf16x8, c);
}

// Operands of one K step of a wave's 128 x 64 sub-tile: 4 u-subtiles and 2 p-subtiles, hi and lo.
struct FwdOps {
    bf16x8 ah[4], al[4], bh[2], bl[2];
};

// Three passes over the 8 accumulators, so consecutive MFMAs never share an accumulator.
template <bool X3>
__device__ __forceinline__ void fwd_mfma(const FwdOps &o, f32x16 (&acc)[4][2]) {
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
            acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(o.ah[a], o.bh[b], acc[a][b], 0, 0, 0);
    if (X3) {
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
                acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(o.ah[a], o.bl[b], acc[a][b], 0, 0, 0);
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
                acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(o.al[a], o.bh[b], acc[a][b], 0, 0, 0);
    }
}

// Both K steps of a chunk.  The operand reads are issued in the order of first use (hi of B, hi of
// A, lo of B, lo of A; step 0, then step 1), the first four operands ahead of the first MFMA and one
// more after each of the next 20 MFMAs, so that every MFMA waits only for its own operands and the
// LDS latency of the later reads hides behind the matrix work.  (Issuing all reads first would make
// the first MFMA wait for most of them: the LDS counter that guards them counts at most 15.)
template <bool X3>
__device__ __forceinline__ void fwd_mma(const char *buf, const OpBase &ox, const OpBase &oy, f32x16 (&acc)[4][2]) {
    static_assert(FKB == 32 && FROW * 16 == 8192, "two K steps per chunk, 16 rows per step");
    const char *xh = buf, *xl = buf + FARR, *yh = buf + 2 * FARR, *yl = buf + 3 * FARR;
    FwdOps o[2];
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) {
#pragma unroll
        for (int b = 0; b < 2; ++b) o[ks].bh[b] = load_opT(yh, oy, b, ks);
#pragma unroll
        for (int a = 0; a < 4; ++a) o[ks].ah[a] = load_opT(xh, ox, a, ks);
        if (X3) {
#pragma unroll
            for (int b = 0; b < 2; ++b) o[ks].bl[b] = load_opT(yl, oy, b, ks);
#pragma unroll
            for (int a = 0; a < 4; ++a) o[ks].al[a] = load_opT(xl, ox, a, ks);
        }
    }
    fwd_mfma<X3>(o[0], acc);
    fwd_mfma<X3>(o[1], acc);
    if (X3) {
        __builtin_amdgcn_sched_group_barrier(0x100, 8, 0);
#pragma unroll
        for (int i = 0; i < 20; ++i) {
            __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
            __builtin_amdgcn_sched_group_barrier(0x100, 2, 0);
        }
        __builtin_amdgcn_sched_group_barrier(0x008, 28, 0);
    } else {
        __builtin_amdgcn_sched_group_barrier(0x100, 8, 0);
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
            __builtin_amdgcn_sched_group_barrier(0x100, 2, 0);
        }
        __builtin_amdgcn_sched_group_barrier(0x008, 8, 0);
    }
}


// ------------------------------------------------------------------------------------------------
// Forward, one wave per SIMD: 256 threads = 4 waves; wave w owns the 128 x 128 output sub-tile
// (u-half w / 2, p-half w % 2) with 16 accumulator tiles (256 accumulator registers).  Every wave
// both generates and contracts: while it contracts chunk c from one LDS buffer, its threads
// generate one X run and one Y run of chunk c + 1 into the other, the generator's VALU work issued
// in the shadow of the MFMAs of the same instruction stream.  One barrier per chunk.
// ------------------------------------------------------------------------------------------------

// The 16 operands of one K step of a 128 x 128 sub-tile.
struct FwdOps1 {
    bf16x8 ah[4], al[4], bh[4], bl[4];
};

// One run of 32 basis values generated in stages spread over the MFMA slots of the chunk, so that
// its VALU work interleaves with the matrix work.  Stage map: 0 starts both recurrences from the
// run's seeds and gives the first two values; 1-30 one value each; the hi/lo split of value pair q
// in two halves at stages 2q + 1 and 2q + 2; the four 16-byte segments (hi and lo) complete at stages
// 8, 16, 24, 32 and are stored there (one-product schedule) or half by half by store_half in later
// slots (three-product schedule).
struct RunStages {
    GenRec R;
    Cheb C, S;
    float v[32];
    unsigned h[16], l[16], hah[16], hbh[16];

    // Stage ST of the run starting at frequency u0, block row k, run r, stored into arr_h / arr_l
    // (X3 false: the hi halves alone, stored into arr_h; STORE false: the segment a stage 8, 16, 24
    // or 32 completes is left to a store_seg call in a later slot).
    template <int ST, bool X3 = true, bool STORE = true>
    __device__ __forceinline__ void stage(int u0, char *arr_h, char *arr_l, int k, int r) {
        constexpr int st = ST;
        // split of pair q: hi at stage 2q + 1, lo at 2q + 2
        constexpr bool HI = st >= 1 && st <= 32 && ((st - 1) & 1) == 0, LO = st >= 1 && st <= 32 && !HI;
        constexpr int q = (st - 1) >> 1;
        if constexpr (X3 && HI) {
            // The pack goes first, ahead of the recurrence step: its result may be read only two wait
            // states later, and with the step in between the shift and mask below need no s_nop.
            h[q] = pack_bf16(v[2 * q], v[2 * q + 1]);
            asm("" : "+v"(h[q]));   // keeps the shift below on h (else it re-converts v[2q] alone)
            __builtin_amdgcn_sched_barrier(0);
        }
        if constexpr (st == 0) {
            start_run(R, C, S);
            v[0] = C.f * S.f;
            if (u0 == 0) v[0] = R.size;
            v[1] = C.next1() * S.next1();
        } else if constexpr (st <= 30) {
            v[st + 1] = C.next1() * S.next1();
        }
        if constexpr (X3 && HI) {
            __builtin_amdgcn_sched_barrier(0);
            hah[q] = h[q] << 16;
            hbh[q] = h[q] & 0xffff0000u;
            // opaque, so that register allocation does not recompute them in the next stage's slot
            asm("" : "+v"(hah[q]), "+v"(hbh[q]));
        } else if constexpr (HI) {
            h[q] = pack_bf16(v[2 * q], v[2 * q + 1]);
        } else if constexpr (X3 && LO) {
            l[q] = split_lo(v[2 * q], v[2 * q + 1], hah[q], hbh[q]);
        }
        if constexpr (STORE && st >= 8 && (st & 7) == 0)
            this->template store_seg<((st - 8) >> 3), X3>(arr_h, arr_l, k, r);
    }
    // Segment M (values 8M .. 8M + 7, complete after stage 8M + 8) into arr_h (and arr_l).
    template <int M, bool X3 = true>
    __device__ __forceinline__ void store_seg(char *arr_h, char *arr_l, int k, int r) {
        *(u32x4 *)(arr_h + fswz(k, 4 * r + M)) = u32x4{h[4 * M], h[4 * M + 1], h[4 * M + 2], h[4 * M + 3]};
        if constexpr (X3)
            *(u32x4 *)(arr_l + fswz(k, 4 * r + M)) = u32x4{l[4 * M], l[4 * M + 1], l[4 * M + 2], l[4 * M + 3]};
    }
    // The hi (HL = 0) or lo (HL = 1) half of segment M into arr.
    template <int M, int HL>
    __device__ __forceinline__ void store_half(char *arr, int k, int r) {
        const unsigned *w = HL ? l : h;
        *(u32x4 *)(arr + fswz(k, 4 * r + M)) = u32x4{w[4 * M], w[4 * M + 1], w[4 * M + 2], w[4 * M + 3]};
    }
    static constexpr int kStages = 33;
};

// Slots of the run stages in a chunk of 96 MFMA slots: the X run's stages spread over slots 0-40,
// the Y run's over slots 41-81 (stage s at slot offset floor(41 s / 33)), so that no slot holds more
// than one stage and the last store precedes the chunk's barrier after slot 83.
constexpr int kRunSlots = 41;
constexpr int run_stage_at(int slot) {
    for (int st = 0; st < RunStages::kStages; ++st)
        if (st * kRunSlots / RunStages::kStages == slot) return st;
    return -1;
}
static_assert((RunStages::kStages - 1) * kRunSlots / RunStages::kStages < kRunSlots, "stage plan");
// Slots of the 16-byte stores of the three-product chunk, [run (X, Y)][segment][hi, lo]: one store in
// each stage-free slot from the one after the stage completing the segment on (the X run's slots
// 10-40 and 46, the Y run's 51-76), the Y run's last segment in slots 81 and 82, so that the barrier's
// wait for the stores (after slot 83) does not wait for stores issued in the slot before it.
constexpr int kFwdStoreSlot[2][4][2] = {{{10, 15}, {20, 25}, {30, 35}, {40, 46}},
                                        {{51, 56}, {61, 66}, {71, 76}, {81, 82}}};
constexpr int kFwdBarrier = 83;   // the chunk's barrier follows this slot
constexpr bool fwd1_stores_ok() {
    for (int run = 0; run < 2; ++run)
        for (int m = 0; m < 4; ++m)
            for (int hl = 0; hl < 2; ++hl) {
                const int sl = kFwdStoreSlot[run][m][hl], done = run * kRunSlots + (8 * m + 8) * kRunSlots / RunStages::kStages;
                const int off = sl - run * kRunSlots;
                if (sl <= done || sl > kFwdBarrier || (off >= 0 && off < kRunSlots && run_stage_at(off) >= 0)) return false;
                if (run == 0 && sl >= kRunSlots && run_stage_at(sl - kRunSlots) >= 0) return false;
            }
    return true;
}
static_assert(fwd1_stores_ok(), "store plan");

// LDS layout of the one-wave forward: the hi and lo arrays of both buffers interleaved,
// [Xh0 Xh1 Xl0 Xl1 | Yh0 Yh1 Yl0 Yl1], 16 KB each, so that with one lane base for the X arrays
// and one (64 KB further) for the Y arrays every operand read of either buffer is the base plus
// an immediate offset below 64 KB.
constexpr int F1_XH(int b) { return b * FARR; }
constexpr int F1_XL(int b) { return (2 + b) * FARR; }
constexpr int F1_YH(int b) { return (4 + b) * FARR; }
constexpr int F1_YL(int b) { return (6 + b) * FARR; }

// Operand OP (0..15) of K step KS of buffer B in first-use order: Ah0, Bh0..3, Ah1..3, Bl0..3,
// Al0..3 (oy carries the 64 KB offset of the Y arrays).
template <int KS, int OP, int B>
__device__ __forceinline__ void fwd1_read(const char *smem, const OpBase &ox, const OpBase &oy, FwdOps1 &o) {
    const char *xh = smem + F1_XH(B), *xl = smem + F1_XL(B);
    const char *yh = smem + F1_YH(B) - F1_YH(0), *yl = smem + F1_YL(B) - F1_YH(0);
    if constexpr (OP == 0) o.ah[0] = load_opT(xh, ox, 0, KS);
    else if constexpr (OP < 5) o.bh[OP - 1] = load_opT(yh, oy, OP - 1, KS);
    else if constexpr (OP < 8) o.ah[OP - 4] = load_opT(xh, ox, OP - 4, KS);
    else if constexpr (OP < 12) o.bl[OP - 8] = load_opT(yl, oy, OP - 8, KS);
    else o.al[OP - 12] = load_opT(xl, ox, OP - 12, KS);
}

// MFMA I (0..47) of one K step: pass hi*hi, then hi*lo, then lo*hi, each over the 16 accumulator
// tiles a-major, so consecutive MFMAs never share an accumulator.
template <int I>
__device__ __forceinline__ void fwd1_mfma(const FwdOps1 &o, f32x16 (&acc)[4][4]) {
    constexpr int pass = I >> 4, a = (I >> 2) & 3, b = I & 3;
    const bf16x8 A = pass == 2 ? o.al[a] : o.ah[a];
    const bf16x8 B = pass == 1 ? o.bl[b] : o.bh[b];
    acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A, B, acc[a][b], 0, 0, 0);
}

struct Fwd1Ctx {
    char *smem;
    const OpBase &ox, &oy;
    f32x16 (&acc)[4][4];
    RunStages &gx, &gy;            // generator of the next chunk (records of the next chunk)
    FwdOps1 &o0, &o1;
    int ux, uy, k, r;
};

// Operand reads are placed in the slots that hold no generator stage (a stage issues about six
// VALU instructions, which one wave issues beside a 32-cycle MFMA at little cost; a stage slot with
// two LDS reads on top stretches the MFMA slot).  Step-0 operands 0-11 of the next chunk are read in
// slots 84-95, after the chunk's barrier, and operands 12-15 of the chunk itself in its stage-free
// slots 10, 25, 30 and 35; the step-1 operands in the stage-free slots 5-76, beside at most one
// store, two per slot where the deadlines crowd.  Every read lands at least six slots before its
// operand's first use.
constexpr int kFwdRead1Slot[16] = {5, 5, 10, 15, 20, 25, 40, 46, 46, 51, 51, 56, 61, 66, 71, 76};
constexpr int fwd1_read0_at(int op) { return op < 12 ? kFwdBarrier + 1 + op : op == 12 ? 10 : op == 13 ? 25 : op == 14 ? 30 : 35; }
template <int OP>
constexpr int fwd1_read0_slot() { return fwd1_read0_at(OP); }
template <int OP>
constexpr int fwd1_read1_slot() { return kFwdRead1Slot[OP]; }
// First use of operand OP in a K step (MFMA order of fwd1_mfma: ah[a] at 4a, bh[b] at b, bl[b] at
// 16 + b, al[a] at 32 + 4a).
constexpr int fwd1_first_use(int op) {
    return op == 0 ? 0 : op < 5 ? op - 1 : op < 8 ? 4 * (op - 4) : op < 12 ? 16 + op - 8 : 32 + 4 * (op - 12);
}
constexpr bool fwd1_reads_ok() {
    for (int op = 0; op < 16; ++op) {
        const int s1 = kFwdRead1Slot[op];
        if (s1 < kRunSlots ? run_stage_at(s1) >= 0 : run_stage_at(s1 - kRunSlots) >= 0) return false;
        if (s1 + 6 > 48 + fwd1_first_use(op)) return false;
        const int s0 = op < 12 ? fwd1_read0_at(op) - 96 : fwd1_read0_at(op);
        if (s0 >= 0 && run_stage_at(s0) >= 0) return false;
        if (s0 + 6 > fwd1_first_use(op)) return false;
    }
    return true;
}
static_assert(fwd1_reads_ok(), "read plan");

template <int I, int B, int... OP>
__device__ __forceinline__ void fwd1_reads0_at(Fwd1Ctx &c, std::integer_sequence<int, OP...>) {
    ((I == fwd1_read0_slot<OP>() ? fwd1_read<0, OP, B>(c.smem, c.ox, c.oy, c.o0) : void()), ...);
}
template <int I, int B, int... OP>
__device__ __forceinline__ void fwd1_reads1_at(Fwd1Ctx &c, std::integer_sequence<int, OP...>) {
    ((I == fwd1_read1_slot<OP>() ? fwd1_read<1, OP, B>(c.smem, c.ox, c.oy, c.o1) : void()), ...);
}

// The stores of slot I into buffer N (S = 8 run + 2 segment + half).
template <int I, int N, int... S>
__device__ __forceinline__ void fwd1_stores_at(Fwd1Ctx &c, std::integer_sequence<int, S...>) {
    ((I == kFwdStoreSlot[S >> 3][(S >> 1) & 3][S & 1]
          ? (S < 8 ? c.gx.template store_half<(S >> 1) & 3, S & 1>(c.smem + ((S & 1) ? F1_XL(N) : F1_XH(N)), c.k, c.r)
                   : c.gy.template store_half<(S >> 1) & 3, S & 1>(c.smem + ((S & 1) ? F1_YL(N) : F1_YH(N)), c.k, c.r))
          : void()),
     ...);
}

// Slot I of a chunk that contracts buffer B and generates into buffer 1 - B.
template <int I, int B>
__device__ __forceinline__ void fwd1_slot(Fwd1Ctx &c) {
    constexpr int N = 1 - B;
    if constexpr (I < 48) fwd1_mfma<I>(c.o0, c.acc);
    else fwd1_mfma<I - 48>(c.o1, c.acc);
    // The records this chunk's runs start from were fetched a chunk ago, the next chunk's (eight
    // loads) since: one wait for the older ones here, in the compiler's own instruction so that it
    // needs no wait of its own at each record's first use.
    if constexpr (I == 0) {
        __builtin_amdgcn_s_waitcnt(0x0F78);   // vmcnt(8)
        __builtin_amdgcn_sched_barrier(0);
    }
    fwd1_reads1_at<I, B>(c, std::make_integer_sequence<int, 16>{});
    constexpr int XS = I < kRunSlots ? run_stage_at(I) : -1;
    constexpr int YS = I >= kRunSlots && I < 2 * kRunSlots ? run_stage_at(I - kRunSlots) : -1;
    if constexpr (XS >= 0) c.gx.template stage<XS, true, false>(c.ux, c.smem + F1_XH(N), c.smem + F1_XL(N), c.k, c.r);
    if constexpr (YS >= 0) c.gy.template stage<YS, true, false>(c.uy, c.smem + F1_YH(N), c.smem + F1_YL(N), c.k, c.r);
    fwd1_stores_at<I, N>(c, std::make_integer_sequence<int, 16>{});
    // The generator's last store is in slot 82 at the latest: after the barrier the next chunk's
    // tiles are complete (its first step-0 operands are read in the following slots, well before the
    // next chunk's first MFMA) and this chunk's buffer is free for the next chunk's generator.
    static_assert(2 * kRunSlots - 1 <= kFwdBarrier && kFwdBarrier + 12 == 95, "slot plan");
    if constexpr (I == kFwdBarrier) lds_barrier();
    if constexpr (I > kFwdBarrier) fwd1_reads0_at<I, N>(c, std::make_integer_sequence<int, 12>{});
    if constexpr (I <= 35) fwd1_reads0_at<I, B>(c, std::make_integer_sequence<int, 16>{});
    __builtin_amdgcn_sched_barrier(0);
}

template <int B, int... I>
__device__ __forceinline__ void fwd1_slots(Fwd1Ctx &c, std::integer_sequence<int, I...>) {
    (fwd1_slot<I, B>(c), ...);
}

// One chunk: contract buffer B into acc while generating the next chunk's X and Y runs into
// buffer 1 - B.  96 slots of one MFMA each; the X run's stages spread over slots 0-40, the Y run's
// over slots 41-81, the hi and lo halves of each run segment stored in stage-free slots after the
// stage completing it (kFwdStoreSlot); the operand reads in the stage-free slots too
// (fwd1_read0_slot, fwd1_read1_slot); the chunk's one barrier follows slot 83.
template <int B>
__device__ __forceinline__ void fwd1_chunk(char *smem, const OpBase &ox, const OpBase &oy, f32x16 (&acc)[4][4],
                                           RunStages &gx, RunStages &gy, FwdOps1 &o0, int ux, int uy, int k,
                                           int r) {
    FwdOps1 o1;
    Fwd1Ctx c{smem, ox, oy, acc, gx, gy, o0, o1, ux, uy, k, r};
    fwd1_slots<B>(c, std::make_integer_sequence<int, 96>{});
}

// One-product chunk (plain bf16, and the one-product tiles of the mixed split): 2 K steps of 16
// MFMA slots (hi*hi over the 16 accumulator tiles, a-major).  Step-1 operands are read at slots 4-11;
// the 33 stages (hi halves only) of the X run and of the Y run spread together over slots 0-27,
// so that every slot holds independent recurrence chains of both runs (one run's stages depend on
// each other, and a slot holding two of them would wait for the VALU latency in between); the
// barrier follows slot 27; the next chunk's first five step-0 operands are read in slots 28-31 and
// the other three in slots 0-2 of their own chunk, each before its first use.
constexpr int kPlainRunSlots = 28;
constexpr int plain_stage_slot(int st) { return st * kPlainRunSlots / RunStages::kStages; }
static_assert(plain_stage_slot(RunStages::kStages - 1) < kPlainRunSlots, "plain stage plan");

template <int I, int N, int... S>
__device__ __forceinline__ void fwd1p_stages(Fwd1Ctx &c, std::integer_sequence<int, S...>) {
    ((plain_stage_slot(S) == I ? (c.gx.template stage<S, false>(c.ux, c.smem + F1_XH(N), nullptr, c.k, c.r),
                                  c.gy.template stage<S, false>(c.uy, c.smem + F1_YH(N), nullptr, c.k, c.r))
                               : void()), ...);
}

template <int I, int B>
__device__ __forceinline__ void fwd1p_slot(Fwd1Ctx &c) {
    constexpr int N = 1 - B;
    if constexpr (I < 16) fwd1_mfma<I>(c.o0, c.acc);
    else fwd1_mfma<I - 16>(c.o1, c.acc);
    if constexpr (I == 0) {   // the runs' records, as in the three-product chunk
        __builtin_amdgcn_s_waitcnt(0x0F78);   // vmcnt(8)
        __builtin_amdgcn_sched_barrier(0);
    }
    if constexpr (I >= 4 && I < 12) fwd1_read<1, I - 4, B>(c.smem, c.ox, c.oy, c.o1);
    if constexpr (I < kPlainRunSlots) fwd1p_stages<I, N>(c, std::make_integer_sequence<int, RunStages::kStages>{});
    if constexpr (I == kPlainRunSlots - 1) lds_barrier();
    if constexpr (I >= 28 && I <= 30) fwd1_read<0, I - 28, N>(c.smem, c.ox, c.oy, c.o0);
    if constexpr (I == 31) {
        fwd1_read<0, 3, N>(c.smem, c.ox, c.oy, c.o0);
        fwd1_read<0, 4, N>(c.smem, c.ox, c.oy, c.o0);
    }
    if constexpr (I <= 2) fwd1_read<0, 5 + I, B>(c.smem, c.ox, c.oy, c.o0);
    __builtin_amdgcn_sched_barrier(0);
}

template <int B, int... I>
__device__ __forceinline__ void fwd1p_slots(Fwd1Ctx &c, std::integer_sequence<int, I...>) {
    (fwd1p_slot<I, B>(c), ...);
}

template <bool X3, int B>
__device__ __forceinline__ void fwd1_chunk_any(char *smem, const OpBase &ox, const OpBase &oy, f32x16 (&acc)[4][4],
                                               RunStages &gx, RunStages &gy, FwdOps1 &o0, int ux, int uy, int k,
                                               int r) {
    if constexpr (X3) {
        fwd1_chunk<B>(smem, ox, oy, acc, gx, gy, o0, ux, uy, k, r);
    } else {
        FwdOps1 o1;
        Fwd1Ctx c{smem, ox, oy, acc, gx, gy, o0, o1, ux, uy, k, r};
        fwd1p_slots<B>(c, std::make_integer_sequence<int, 32>{});
    }
}

// Step-0 operands of the first chunk that the loop expects already read: 0-11 for the three-product
// schedule, 0-4 for the one-product one.
template <bool X3, int... OP>
__device__ __forceinline__ void fwd1_prologue_reads(const char *smem, const OpBase &ox, const OpBase &oy, FwdOps1 &o0,
                                                    std::integer_sequence<int, OP...>) {
    (((X3 ? OP < 12 : OP < 5) ? fwd1_read<0, OP, 0>(smem, ox, oy, o0) : void()), ...);
}

// X3: three products per pair (hi*hi, lo*hi, hi*lo); otherwise one (hi*hi).  skip_u x skip_p: the
// tiles of that low-frequency corner are left to another launch (the mixed split contracts them
// with three products); 0 x 0 skips nothing.
template <bool X3>
__global__ __launch_bounds__(256) void k_fwd1_bf16(int64_t n, int Mu, int Mp, const PhaseRec *__restrict__ tx,
                                                   const PhaseRec *__restrict__ ty, const RunSeed *__restrict__ sx,
                                                   const RunSeed *__restrict__ sy, float *__restrict__ part,
                                                   int tiles_p, int64_t chunks, int64_t chunks_per_split, int skip_u,
                                                   int skip_p) {
    __shared__ __attribute__((aligned(16))) char smem[2 * FBUF];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t rows = phase_rows(n);
    int tile;
    int64_t split;
    fwd_tile_split(tile, split);
    if (tile / tiles_p < skip_u && tile % tiles_p < skip_p) return;   // the whole workgroup, before any barrier
    const int tu0 = (tile / tiles_p) * FT, tp0 = (tile % tiles_p) * FT;
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
    OpBase ox, oy;
    ox.init(wu, lane);
    oy.init(wp, lane);
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int rd = 0; rd < 2; ++rd) oy.b[a][rd] += F1_YH(0);

    // Thread tid generates block k = tid % 32 of each chunk, frequencies 32 r .. + 31 of the tile.
    const int kk = tid & 31, rr = tid >> 5;
    const int ux = tu0 + 32 * rr, uy = tp0 + 32 * rr;
    const int runx = ux / 32, runy = uy / 32;
    // the records of chunk `ch` (the tables are padded with zero rows past the last chunk + 2)
    auto recx = [&](int64_t ch) { return load_gen(tx, sx, rows, runx, ch * FKB + kk); };
    auto recy = [&](int64_t ch) { return load_gen(ty, sy, rows, runy, ch * FKB + kk); };
    if (c_begin < c_end) {
        fwd_gen<X3>(recx(c_begin), tu0, smem + F1_XH(0), smem + F1_XL(0), tid);
        fwd_gen<X3>(recy(c_begin), tp0, smem + F1_YH(0), smem + F1_YL(0), tid);
    }
    // Two record sets alternate: the chunk at even offset from c_begin generates from set B and
    // fetches the records of the chunk after next into set A, the chunk at odd offset the reverse.
    // (Past the range: zero records or records of the next split, generated into the idle buffer
    // and never read.)
    RunStages gxA, gyA, gxB, gyB;
    gxB.R = recx(c_begin + 1);
    gyB.R = recy(c_begin + 1);
    lds_barrier();
    FwdOps1 o0;
    fwd1_prologue_reads<X3>(smem, ox, oy, o0, std::make_integer_sequence<int, 14>{});
    // Nothing the prologue loaded may still be in flight at the loop head (the compiler would then
    // wait for every load and LDS read at the first use in each iteration); the wait is the
    // compiler's own instruction, so that its bookkeeping knows.
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_waitcnt(0x0070);   // vmcnt(0) lgkmcnt(0)
    asm volatile("" ::: "memory");
    int64_t c = c_begin;
    for (; c + 1 < c_end; c += 2) {
        gxA.R = recx(c + 2);
        gyA.R = recy(c + 2);
        fwd1_chunk_any<X3, 0>(smem, ox, oy, acc, gxB, gyB, o0, ux, uy, kk, rr);
        gxB.R = recx(c + 3);
        gyB.R = recy(c + 3);
        fwd1_chunk_any<X3, 1>(smem, ox, oy, acc, gxA, gyA, o0, ux, uy, kk, rr);
    }
    if (c < c_end) fwd1_chunk_any<X3, 0>(smem, ox, oy, acc, gxB, gyB, o0, ux, uy, kk, rr);

    float *out = part + (size_t)split * (size_t)Mu * (size_t)Mp;
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int u = tu0 + wu + 32 * a + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                const int p = tp0 + wp + 32 * b + (lane & 31);
                if (u < Mu && p < Mp) out[(size_t)u * Mp + p] = acc[a][b][r];
            }
}

// ================================================================================================
// Backward: G[i][nn] = sum_k A_ik B[k][nn], g_i = sum_nn E_i,nn G[i][nn].
// Kernels: k_bwd1_bf16 (the basis regenerated, one wave per SIMD, three products or one, further
// below) and k_bwd_bf16_st (the store mode of both bf16 types, A read from the stored table, here).
// A (sine differences along the K axis) is held in MFMA operand layout: lane half h = lane / 32
// walks frequencies h * Kh + 8 t (t = 0, 1, ...), so each lane's recurrence (or table row) runs over
// contiguous frequencies.  B is staged per chunk of 32 + 32 frequencies
// (4 K steps) in LDS by direct copies (global memory to LDS, no registers; buffer loads in the
// regenerating kernel, global ones in the store-mode kernel): the global operand is pre-tiled in exactly the
// LDS byte order, one contiguous 64 KB block (hi then lo) per (N tile, chunk), rows of 128 bytes
// whose 16-byte segments are XOR-swizzled by (row / 2) % 8: any 16 consecutive rows then cover all
// 16 bank groups of 16 bytes, so the b128 operand reads are conflict free.
// ================================================================================================
constexpr int BTN = 256;                 // N tile (columns)
constexpr int BKC = 64;                  // K values per chunk (32 from each half)
constexpr int BROW = BKC * 2;            // bytes per LDS row (128)
constexpr int BARR = BTN * BROW;         // bytes per hi or lo array (32 KB)
constexpr int BBUF = 2 * BARR;           // one chunk, hi + lo (64 KB)

// Issue the direct copies of one 64 KB chunk tile: 8 slices of 8 KB, each wave 1 KB per slice.
__device__ __forceinline__ void bwd_copy_b(const unsigned short *__restrict__ gtile, char *buf, int tid) {
    const int wave = tid >> 6;
    typedef __attribute__((address_space(3))) void lds_void;
#pragma unroll
    for (int i = 0; i < BBUF / 8192; ++i)
        __builtin_amdgcn_global_load_lds((const void *)((const char *)gtile + i * 8192 + tid * 16),
                                         (lds_void *)(buf + i * 8192 + wave * 1024), 16, 0, 0);
}

// The epilogue basis value of kind EK at frequency nn from the phasors (ca, sa) of nn alpha and
// (cb, sb) of nn beta (alpha = pi c / L, beta = pi sz / (2L)); pil = pi / L.
template <int EK>
__device__ __forceinline__ float ep_value(float ca, float sa, float cb, float sb, int nn, float size, float pil) {
    (void)cb;
    if constexpr (EK == RUN_COSDIFF) return -2.0f * sa * sb;
    else if constexpr (EK == RUN_SINDIFF) return nn == 0 ? size : 2.0f * ca * sb;
    else if constexpr (EK == RUN_COS) return ca;
    else return (float)nn * pil * sa;
}

// Gradient contraction from the stored basis (store mode): G[i][nn] = sum_k S_ik B[k][nn] with S read
// from its table, then the cosine-difference row dot.  512 threads = 8 waves, wave w owning blocks
// i0 + 32 w .. + 31 and all 256 columns of the N tile (8 accumulator tiles).
template <bool X3>
__global__ __launch_bounds__(512) void k_bwd_bf16_st(int64_t n, BwdAxisBf16 ax) {
    __shared__ __attribute__((aligned(16))) char smem[2 * BBUF];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int h = lane >> 5, j = lane & 31;
    // One-dimensional grid, workgroups dealt round-robin over the 8 XCDs: the N tiles of one block
    // tile go to the same XCD at about the same time, so they share its L2 copy of the block tile's
    // table rows.
    const int w = blockIdx.x, xcd = w & 7, slot = w >> 3;
    const int btile = xcd + 8 * (slot / ax.tiles_n);
    const int ntile = slot % ax.tiles_n;
    if (btile >= ax.tiles_b) return;
    const int64_t i0 = (int64_t)btile * 256 + 32 * wave;
    const int n0 = ntile * BTN;
    const int64_t ib = i0 + j;        // this lane's block for the A operand
    const int Q = ax.Kh / 32;         // chunks along K

    f32x16 acc[8];
#pragma unroll
    for (int b = 0; b < 8; ++b)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[b][r] = 0.0f;

    const size_t tile_elems = (size_t)BBUF / 2;      // bf16 elements per chunk tile (hi + lo)
    const unsigned short *gb = ax.B + (size_t)ntile * Q * tile_elems;

    // One K step: B operands (row 32 b + j, logical segment 4 h + s, physical segment XORed with
    // (j / 2) % 8) and the three MFMA passes over the 8 accumulators.
    auto mma_step = [&](const char *cur, int s, const bf16x8 &ah, const bf16x8 &al) {
        const int bseg = ((4 * h + s) ^ ((j >> 1) & 7)) * 16;
        bf16x8 bh[8], bl[8];
#pragma unroll
        for (int b = 0; b < 8; ++b) bh[b] = *(const bf16x8 *)(cur + (32 * b + j) * BROW + bseg);
        if (X3) {
#pragma unroll
            for (int b = 0; b < 8; ++b) bl[b] = *(const bf16x8 *)(cur + BARR + (32 * b + j) * BROW + bseg);
        }
#pragma unroll
        for (int b = 0; b < 8; ++b) acc[b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bh[b], acc[b], 0, 0, 0);
        if (X3) {
#pragma unroll
            for (int b = 0; b < 8; ++b) acc[b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bh[b], acc[b], 0, 0, 0);
#pragma unroll
            for (int b = 0; b < 8; ++b) acc[b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bl[b], acc[b], 0, 0, 0);
        }
    };

    // A from the stored basis table: row ib, frequencies h Kh + 32 q + 8 s + 0..7 for step s of chunk
    // q (rows past n are zero).  The next chunk's operands are requested before its B copies, a whole
    // chunk ahead of their use.
    const unsigned short *rh = ax.tab_h + (size_t)ib * (size_t)ax.tab_ld + h * ax.Kh;
    const unsigned short *rl = ax.tab_l + (size_t)ib * (size_t)ax.tab_ld + h * ax.Kh;
    bf16x8 cah[4], cal[4], nah[4], nal[4];
    auto load_a = [&](int q, bf16x8 (&dh)[4], bf16x8 (&dl)[4]) {
#pragma unroll
        for (int st = 0; st < 4; ++st) {
            dh[st] = *(const bf16x8 *)(rh + 32 * q + 8 * st);
            if (X3) dl[st] = *(const bf16x8 *)(rl + 32 * q + 8 * st);
        }
    };
    load_a(0, cah, cal);
    bwd_copy_b(gb, smem, tid);
    wait_copies();
    __syncthreads();
    for (int q = 0; q < Q; ++q) {
        char *cur = smem + (q & 1) * BBUF, *nxt = smem + ((q & 1) ^ 1) * BBUF;
        if (q + 1 < Q) {
            load_a(q + 1, nah, nal);
            bwd_copy_b(gb + (size_t)(q + 1) * tile_elems, nxt, tid);
        }
#pragma unroll
        for (int st = 0; st < 4; ++st) mma_step(cur, st, cah[st], cal[st]);
        wait_copies();
        __syncthreads();
#pragma unroll
        for (int st = 0; st < 4; ++st) {
            cah[st] = nah[st];
            if (X3) cal[st] = nal[st];
        }
    }

    // Epilogue: lane holds G for rows 8 (r / 4) + 4 h + r % 4 and columns n0 + 32 b + j;
    // E = -2 sin(nn alpha) sin(nn beta) of the epilogue axis, stepped by 32 columns.  Each lane sums
    // its 8 columns of a row in FP32; the 32 lanes of the row add in FP64.
    double rs[16];
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
                sum = fmaf(ep_value<RUN_COSDIFF>(ca0, sa0, cb0, sb0, nn + 32 * b, RE.size, ax.pil), acc[b][r], sum);
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
        double v = rs[r];
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
            if (ibe < n) ax.gpart[(size_t)ntile * (size_t)n + (size_t)ibe] = rs[r];
        }
    }
}

// ------------------------------------------------------------------------------------------------
// Backward, one wave per SIMD (x3): 256 threads = 4 waves; wave w owns blocks i0 + 64 w .. + 63
// (two 32-block subtiles) and all 256 columns of the N tile, 16 accumulator tiles.  Each wave
// generates its A operands in registers one K step ahead, in the shadow of the current step's
// MFMAs; B is read from LDS in the order of first use.  One barrier per chunk, in its last step:
// after it the next chunk's tile (copied a chunk ahead) is read, and the chunk after next is copied
// into the buffer just released.
// ------------------------------------------------------------------------------------------------

// A-operand generator of one 32-block subtile: recurrence state and two fp32 phasors of the current
// frequency, e^{i pi k ta} and e^{i pi k tb}, seeded once in FP64 and advanced by the record's
// 32-frequency phasors at every reseed (no memory access and no FP64 reduction in the K loop; drift
// after 64 jumps ~1e-6), with the values and split halves of the step being generated.  The generator's
// work is cut into pieces of at most three VALU instructions (a value; the FMAs that advance both
// recurrences; one half of a hi/lo split; half of a phasor jump), so that the pieces can be dealt
// over the MFMA slots evenly.
template <int KA>
struct AGen {
    Cheb ca, sb;
    float pac, pas, pbc, pbs, jac, jas, jbc, jbs, sac, sas, sbc, sbs, size0;
    float tj0, tj1;               // phasor jump in flight
    float v[8];
    unsigned hh[4], ll[4], hah[4], hbh[4];

    __device__ __forceinline__ void init(const PhaseRec *__restrict__ tab, int64_t ib, bool valid, int k0) {
        if (valid) {
            const PhaseRec RA = tab[ib];
            seed_phasor(k0, RA.ta, pac, pas);
            seed_phasor(k0, RA.tb, pbc, pbs);
            jac = RA.ca32; jas = RA.sa32; jbc = RA.cb32; jbs = RA.sb32;
            sac = RA.ca; sas = RA.sa; sbc = RA.cb; sbs = RA.sb;
            ca.ch = RA.c2ah; ca.cl = RA.c2al; sb.ch = RA.c2bh; sb.cl = RA.c2bl;
            size0 = RA.size;
        } else {
            pac = pas = pbc = pbs = jac = jas = jbc = jbs = sac = sas = sbc = sbs = size0 = 0.0f;
            ca.ch = ca.cl = sb.ch = sb.cl = 0.0f;
        }
        reseed();
    }
    __device__ __forceinline__ void reseed() {
        ca.f = pac;
        ca.fm = pac * sac + pas * sas;                // cos((k - 1) alpha)
        sb.f = 2.0f * pbs;                            // 2 sin(k beta)
        sb.fm = 2.0f * (pbs * sbc - pbc * sbs);       // 2 sin((k - 1) beta)
    }
    // The phasors advance by 32 frequencies in four pieces: the new cosine of alpha, then its sine
    // (from the old cosine), then the same for beta.
    template <int P>
    __device__ __forceinline__ void jump() {
        if constexpr (P == 0) tj0 = pac * jac - pas * jas;
        else if constexpr (P == 1) { pas = pas * jac + pac * jas; pac = tj0; }
        else if constexpr (P == 2) tj1 = pbc * jbc - pbs * jbs;
        else { pbs = pbs * jbc + pbc * jbs; pbc = tj1; }
    }
    // Value E of the step (frequency k + E) and the first FMA of each recurrence; at k = 0 the
    // sine-difference kind takes the block size (FIRST0: this step starts at frequency 0).
    template <int E, bool FIRST0>
    __device__ __forceinline__ void value1() {
        if constexpr (KA == RUN_COS) {
            v[E] = ca.f;
        } else {
            v[E] = ca.f * sb.f;
            if constexpr (E == 0 && FIRST0) v[0] = size0;
        }
    }
    // The second FMAs: the recurrences advance by one frequency.
    __device__ __forceinline__ void value2() {
        const float nc = fmaf(ca.ch, ca.f, -ca.fm);   // the centre factor: one FMA (Cheb::next1)
        ca.fm = ca.f;
        ca.f = nc;
        if constexpr (KA != RUN_COS) {
            const float ns = fmaf(sb.ch, sb.f, -sb.fm);
            sb.fm = sb.f;
            sb.f = ns;
        }
    }
    template <int M>
    __device__ __forceinline__ void half_hi() {
        hh[M] = pack_bf16(v[2 * M], v[2 * M + 1]);
        asm("" : "+v"(hh[M]));   // keeps the shift below on hh (else v[2M] is converted again)
        hah[M] = hh[M] << 16;
        hbh[M] = hh[M] & 0xffff0000u;
    }
    template <int M>
    __device__ __forceinline__ void half_lo() {
        ll[M] = split_lo(v[2 * M], v[2 * M + 1], hah[M], hbh[M]);
    }
    // One-product contraction: the hi half alone (no lo split follows).
    template <int M>
    __device__ __forceinline__ void pack_hi() { hh[M] = pack_bf16(v[2 * M], v[2 * M + 1]); }
    __device__ __forceinline__ bf16x8 hi() const { return __builtin_bit_cast(bf16x8, u32x4{hh[0], hh[1], hh[2], hh[3]}); }
    __device__ __forceinline__ bf16x8 lo() const { return __builtin_bit_cast(bf16x8, u32x4{ll[0], ll[1], ll[2], ll[3]}); }
};

template <int KA>
struct Bwd1Ctx {
    const char *cur, *nxt;
    char *cpy_dst;                 // released buffer receiving the chunk after next (after the barrier)
    unsigned cpy_off;              // its byte offset in the operand (past the last chunk: the last chunk again)
    char *cpy_dst2;                // buffer receiving the next chunk (the rest of its copies)
    unsigned cpy_off2;             // its byte offset in the operand (past the last chunk: the last chunk again)
    const char *gtile;             // the N tile's operand, Q chunks of 64 KB
    int gbytes;                    // its size
    AGen<KA> (&g)[2];
    bf16x8 (&ah)[2], (&al)[2];     // A operands of the current step
    bf16x8 (&bh)[8], (&bl)[8];     // B operands
    f32x16 (&acc)[2][8];
    int h, j;
    unsigned lane_off;             // this lane's byte offset within a copy slice
    int wave_off;                  // 1024 times the wave's index (uniform)
};

// Copy slice SL (0 .. NSL - 1) of this wave's quarter of the first 4 NSL KB of an operand tile
// (NSL = 16: hi and lo, the whole tile; 8: the hi half): tile bytes NSL wave_off + 1024 SL + 16 lane
// go to the same offset of the LDS buffer (NEXT: the next chunk's tile and buffer, else the chunk
// after next's).  The copy is a buffer load into LDS: the lane's offset in a register, the chunk's
// in a scalar one, and four consecutive slices differ only in the immediate offset, which moves the
// global and the LDS address alike (one M0 value per group of four).  Unlike the global form, which
// the compiler also books as an LDS access and then answers with a full LDS wait at the next use of
// any LDS read, the buffer form counts as a memory load only.
template <int IMM>
__device__ __forceinline__ void bwd1_copy16(const char *gtile, int gbytes, unsigned voff, unsigned soff, char *lds) {
    typedef __attribute__((address_space(3))) void lds_void;
    // raw buffer resource of the N tile's operand (uniform; the compiler keeps one in scalar registers)
    const __amdgpu_buffer_rsrc_t rsrc = __builtin_amdgcn_make_buffer_rsrc((void *)gtile, (short)0, gbytes, 0x00020000);
    __builtin_amdgcn_raw_ptr_buffer_load_lds(rsrc, (lds_void *)lds, 16, voff, soff, IMM, 0);
}
template <int SL, int NSL, bool NEXT, int KA>
__device__ __forceinline__ void bwd1_copy_slice(const Bwd1Ctx<KA> &c) {
    static_assert(NSL % 4 == 0 && SL >= 0 && SL < NSL, "copy slices");
    constexpr int grp = (SL >> 2) * 4096;
    const int part = NSL * c.wave_off + grp;
    bwd1_copy16<(SL & 3) * 1024>(c.gtile, c.gbytes, c.lane_off + NSL * c.wave_off,
                                 (NEXT ? c.cpy_off2 : c.cpy_off) + grp, (NEXT ? c.cpy_dst2 : c.cpy_dst) + part);
}

// A wait for every outstanding LDS operation written with the compiler's own instruction, so that its
// bookkeeping sees the reads complete (the empty asm statements keep memory operations on their side).
__device__ __forceinline__ void counted_lds_wait() {
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_waitcnt(0xC07F);   // lgkmcnt(0); vmcnt and expcnt at their maxima (no wait)
    asm volatile("" ::: "memory");
}

// Copy plan of a chunk whose barrier follows slot BAR.  The four waves' direct copies share the CU's
// memory pipeline, and issued in consecutive slots they slow the waves down (bunched into six slots
// they cost the three-product kernel 1.5 % more than one per slot after the barrier, and one per
// four to eight slots cost 1.5 % less); they are therefore spread out.  A buffer is free from the
// barrier of the chunk that read it, and the tile for chunk q + 2 must have landed by the barrier of
// chunk q + 1: slices 0 and 1 go in slots BAR + 1 and BAR + 1 + D of chunk q (into the buffer that
// chunk q released), slices 2 .. NSL - 1 in slots 0, D, 2 D, ... of chunk q + 1 (into its next
// buffer), well before that chunk's barrier.
template <int BAR, int D>
constexpr int bwd1_copy_after(int slot) { return slot == BAR + 1 ? 0 : slot == BAR + 1 + D ? 1 : -1; }
template <int NSL, int D>
constexpr int bwd1_copy_next(int slot) { return slot % D == 0 && slot / D + 2 < NSL ? slot / D + 2 : -1; }
// The three-product chunk places them by its LDS waits instead (slots 32, 48, 80, 96, 128 and 144 of
// the chunk, the first uses of the lo and hi B reads): slices 2 .. 15 right after such a wait and at
// least 15 slots before the next one, slices 0 and 1 after an explicit wait for the next chunk's hi B
// reads, at slots 188 and 190, so that the next chunk's first MFMAs need no wait at all.  (The plan
// dates from copies issued as global loads into LDS, which the compiler also books as LDS accesses,
// turning every later LDS wait into a wait for all of them; the buffer form it uses now counts as a
// memory load only, and the plan measured no worse with it.)
constexpr int kBwd1CopyNext[14] = {1, 5, 9, 13, 49, 53, 57, 61, 97, 101, 105, 109, 145, 149};
constexpr int bwd1x3_copy_next(int slot) {
    for (int k = 0; k < 14; ++k)
        if (kBwd1CopyNext[k] == slot) return k + 2;
    return -1;
}
constexpr int bwd1x3_copy_after(int slot) { return slot == 188 ? 0 : slot == 190 ? 1 : -1; }

// Compile-time check of the copy plans against the chunk's reads and barrier, for 1 to 6 chunks.
// Copies land at the barrier's wait (each wave waits for its own, then all meet), and waves are
// ordered only by barriers, so: every read of a buffer finds there the whole operand tile of the
// chunk it expects (NSL slices), none of it still in flight, and a copy writes a buffer only when
// every read of that buffer lies at or before the last barrier.  Reads: three products, lo B at
// slots 16-23 and hi B at slots 32-39 of each step (the next chunk's hi B, from the other buffer, in
// step 3), barrier after slot 175; one product, hi B at slots 8-15 of each step (the next chunk's in
// step 3), barrier after slot 55.
template <bool X3>
constexpr bool bwd1_copy_plan_ok() {
    constexpr int NS = X3 ? 192 : 64, BAR = X3 ? 175 : 55, NSL = X3 ? 16 : 8, STEP = X3 ? 48 : 16;
    for (int Q = 1; Q <= 6; ++Q) {
        int have[2][16] = {}, src[2][16] = {};
        bool pend[2][16] = {};
        int lastread[2] = {-1, -1}, lastbar = -1;
        for (int b = 0; b < 2; ++b)
            for (int sl = 0; sl < 16; ++sl) have[b][sl] = -1;
        for (int sl = 0; sl < NSL; ++sl) have[0][sl] = 0;       // prologue: chunk 0,
        if (Q > 1) have[1][0] = have[1][1] = 1;                 // the first two slices of chunk 1
        for (int q = 0; q < Q; ++q) {
            const int cur = q & 1, nxt = cur ^ 1;
            const int after = q + 2 < Q - 1 ? q + 2 : Q - 1, next = q + 1 < Q - 1 ? q + 1 : Q - 1;
            for (int i = 0; i < NS; ++i) {
                const int g = q * NS + i, s = i / STEP, t = i % STEP;
                const int ca = X3 ? bwd1x3_copy_after(i) : bwd1_copy_after<55, 4>(i);
                const int cn = X3 ? bwd1x3_copy_next(i) : bwd1_copy_next<8, 4>(i);
                if (ca >= 0) {
                    if (lastread[cur] > lastbar) return false;
                    pend[cur][ca] = true;
                    src[cur][ca] = after;
                }
                if (cn >= 0) {
                    if (lastread[nxt] > lastbar) return false;
                    pend[nxt][cn] = true;
                    src[nxt][cn] = next;
                }
                int rb = -1, need = 0;   // buffer read in this slot and the chunk it must hold
                if (X3 && t >= 16 && t < 24) rb = cur, need = q;
                if (t >= (X3 ? 32 : 8) && t < (X3 ? 40 : 16)) rb = s < 3 ? cur : nxt, need = s < 3 ? q : q + 1;
                if (rb >= 0) {
                    if (need < Q)
                        for (int sl = 0; sl < NSL; ++sl)
                            if (pend[rb][sl] || have[rb][sl] != need) return false;
                    lastread[rb] = g;
                }
                if (i == BAR) {
                    for (int b = 0; b < 2; ++b)
                        for (int sl = 0; sl < 16; ++sl)
                            if (pend[b][sl]) have[b][sl] = src[b][sl], pend[b][sl] = false;
                    lastbar = g;
                }
            }
        }
    }
    return true;
}
static_assert(bwd1_copy_plan_ok<true>() && bwd1_copy_plan_ok<false>(), "copy plan hazard");

// B operand of column tile b, K step s of a chunk buffer: row 32 b + j, logical segment 4 h + s,
// physical segment XORed with (j / 2) % 8.
__device__ __forceinline__ bf16x8 bwd1_readb(const char *buf, int hl, int b, int s, int h, int j) {
    const int bseg = ((4 * h + s) ^ ((j >> 1) & 7)) * 16;
    return *(const bf16x8 *)(buf + hl * BARR + (32 * b + j) * BROW + bseg);
}

// Generator work of slot T (0..47) of a step, for the A operands of the following step (GS: the
// step whose slots these are; FIRST0: the generated step starts at frequency 0).  Value u = 2 e + a
// (e: frequency within the step, a: subtile) takes slots 3u (the value and first FMAs) and 3u + 1
// (second FMAs).  Value pair m of subtile a is complete at slot 3 u2 with u2 = 4 m + 2 + a; its hi
// half is split off at 3 u2 + 2 and, for m < 3, its lo half at 3 (u2 + 2) + 2.  The lo halves of
// pair 3 fall into slots 2 and 5 of the next step, whose lo operands are assembled at slot 6 and
// first used at slot 16; the hi operands are assembled at slot 47.  In step 0 the phasor jump
// takes the second-FMA slots 1-22; in step 2 each subtile is reseeded from its phasors after its
// last value of the chunk.
template <int KA, int GS, bool FIRST0, int T>
__device__ __forceinline__ void bwd1_gen(Bwd1Ctx<KA> &c) {
    constexpr int u = T / 3, ph = T % 3;
    constexpr int a = u & 1, e = u >> 1;
    if constexpr (ph == 0) c.g[a].template value1<e, FIRST0>();
    if constexpr (ph == 1) c.g[a].value2();
    if constexpr (ph == 2) {
        // hi halves at u = 4 m + 2 + a, lo halves (m < 3) at u = 4 m + 4 + a, lo of pair 3 at u = a
        constexpr int r4 = u & 3;
        if constexpr (r4 >= 2) c.g[r4 - 2].template half_hi<(u >> 2)>();
        else if constexpr (u >= 4) c.g[r4].template half_lo<(u >> 2) - 1>();
        else c.g[r4].template half_lo<3>();
    }
    if constexpr (GS == 0 && ph == 1 && u < 8) c.g[u >> 2].template jump<u & 3>();
    if constexpr (GS == 2 && T == 45) c.g[0].reseed();
    if constexpr (GS == 2 && T == 47) c.g[1].reseed();
}

// Slot I (0..191) of a chunk: one MFMA, the B reads, copies and generator work assigned to it, then
// a scheduling fence.  MFMA order within a step: pass (hi*hi, lo*hi, hi*lo), column tile b,
// subtile a.
template <int KA, int I>
__device__ __forceinline__ void bwd1_slot(Bwd1Ctx<KA> &c) {
    constexpr int s = I / 48, t = I % 48;
    constexpr int pass = t / 16, b = (t % 16) / 2, a = t % 2;
    {
        const bf16x8 A = pass == 1 ? c.al[a] : c.ah[a];
        const bf16x8 B = pass == 2 ? c.bl[b] : c.bh[b];
        c.acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A, B, c.acc[a][b], 0, 0, 0);
    }
    // The MFMA goes first in its slot: after the chunk's barrier the slot's B read would otherwise be
    // issued ahead of it, and the wait for the MFMA's own operand then covers that fresh read too.
    __builtin_amdgcn_sched_barrier(0);
    // lo B of this step in the first half of the lo*hi pass, hi B of the next step in the first half
    // of the hi*lo pass: each read lands at least 8 slots before its first use, so that even a full
    // LDS wait (the compiler's while direct copies are in flight) finds them complete.
    if constexpr (t >= 16 && t < 24) c.bl[t - 16] = bwd1_readb(c.cur, 1, t - 16, s, c.h, c.j);
    if constexpr (s == 3 && t == 31) {
        // all reads of this chunk's buffer are done and the next chunk's copies have landed
        wait_copies();
        lds_barrier();
    }
    if constexpr (t >= 32 && t < 40) {
        constexpr int bb = t - 32;
        if constexpr (s < 3) c.bh[bb] = bwd1_readb(c.cur, 0, bb, s + 1, c.h, c.j);
        else c.bh[bb] = bwd1_readb(c.nxt, 0, bb, 0, c.h, c.j);
    }
    {
        // copies (unconditional, so that the chunk stays one basic block: past the end the last
        // chunk is copied again into a buffer that is not read any more)
        constexpr int ca = bwd1x3_copy_after(I), cn = bwd1x3_copy_next(I);
        if constexpr (I == 188) counted_lds_wait();
        if constexpr (ca >= 0) bwd1_copy_slice<ca, 16, false>(c);
        if constexpr (cn >= 0) bwd1_copy_slice<cn, 16, true>(c);
    }
    bwd1_gen<KA, s, false, t>(c);
    if constexpr (t == 6) {
#pragma unroll
        for (int aa = 0; aa < 2; ++aa) c.al[aa] = c.g[aa].lo();
    }
    if constexpr (t == 47) {
#pragma unroll
        for (int aa = 0; aa < 2; ++aa) c.ah[aa] = c.g[aa].hi();
    }
    __builtin_amdgcn_sched_barrier(0);
}

// One-product chunk (plain bf16, and the one-product N tiles of the mixed split): 4 steps of 16 slots,
// slot t of a step holding MFMA (column tile t / 2, subtile t % 2) and the whole generator work of
// value u = t of the following step (its value and both FMAs of the recurrences, and the hi half of
// the pair it completes); the phasor jump takes slots 0-7 of step 0, the reseeds follow the last
// value of each subtile in step 2.  Next step's hi B is read at slots 8-15, at least 8 slots ahead
// of its first use and after the current step's last use of the same register; the barrier moves
// to slot 7 of step 3; the copies (hi halves only) follow bwd1_copy_after and bwd1_copy_next.
template <int KA, int I>
__device__ __forceinline__ void bwd1_slot_plain(Bwd1Ctx<KA> &c) {
    constexpr int s = I / 16, t = I % 16;
    constexpr int b = t / 2, a = t % 2;
    c.acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(c.ah[a], c.bh[b], c.acc[a][b], 0, 0, 0);
    if constexpr (s == 3 && t == 7) {
        wait_copies();
        lds_barrier();
    }
    if constexpr (t >= 8) {
        constexpr int bb = t - 8;
        if constexpr (s < 3) c.bh[bb] = bwd1_readb(c.cur, 0, bb, s + 1, c.h, c.j);
        else c.bh[bb] = bwd1_readb(c.nxt, 0, bb, 0, c.h, c.j);
    }
    {
        constexpr int ca = bwd1_copy_after<55, 4>(I), cn = bwd1_copy_next<8, 4>(I);
        static_assert(55 + 1 + 4 < 64 && 4 * 5 < 55 - 24, "copy plan");
        if constexpr (ca >= 0) bwd1_copy_slice<ca, 8, false>(c);
        if constexpr (cn >= 0) bwd1_copy_slice<cn, 8, true>(c);
    }
    {
        constexpr int u = t, ga = u & 1, e = u >> 1;
        c.g[ga].template value1<e, false>();
        c.g[ga].value2();
        if constexpr ((u & 3) >= 2) c.g[ga].template pack_hi<(u >> 2)>();
        if constexpr (s == 0 && u < 8) {
            c.g[u >> 2].template jump<(u & 3)>();
        }
        if constexpr (s == 2 && u == 14) c.g[0].reseed();
        if constexpr (s == 2 && u == 15) c.g[1].reseed();
    }
    if constexpr (t == 15) {
#pragma unroll
        for (int aa = 0; aa < 2; ++aa) c.ah[aa] = c.g[aa].hi();
    }
    __builtin_amdgcn_sched_barrier(0);
}

template <bool X3, int KA, int... I>
__device__ __forceinline__ void bwd1_slots(Bwd1Ctx<KA> &c, std::integer_sequence<int, I...>) {
    if constexpr (X3) (bwd1_slot<KA, I>(c), ...);
    else (bwd1_slot_plain<KA, I>(c), ...);
}

template <int KA, bool FIRST0, int... T>
__device__ __forceinline__ void bwd1_gen_all(Bwd1Ctx<KA> &c, std::integer_sequence<int, T...>) {
    (bwd1_gen<KA, 1, FIRST0, T>(c), ...);
}


// X3: three products per pair (hi*hi, lo*hi, hi*lo); otherwise one (hi*hi).
template <bool X3, int KA, int E1, int E2>
__global__ __launch_bounds__(256) void k_bwd1_bf16(int64_t n, BwdAxisBf16 ax) {
    __shared__ __attribute__((aligned(16))) char smem[2 * BBUF];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int h = lane >> 5, j = lane & 31;
    const int btile = blockIdx.x, ntile = blockIdx.y + ax.nt0;
    const int64_t i0 = (int64_t)btile * 256 + 64 * wave;
    const int n0 = ntile * BTN;
    const int Q = ax.Kh / 32;
    const size_t tile_bytes = (size_t)BBUF;
    const char *gb = (const char *)ax.B + (size_t)ntile * Q * tile_bytes;

    AGen<KA> g[2];
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

    // Prologue: copies of chunk 0 and of the first two slices of chunk 1 (the rest of chunk 1 is
    // copied in chunk 0's slots), A of step 0 of chunk 0, hi B of step 0.
    typedef __attribute__((address_space(3))) void lds_void;
#pragma unroll
    for (int sl = 0; sl < BBUF / 4096; ++sl)
        __builtin_amdgcn_global_load_lds((const void *)(gb + sl * 4096 + tid * 16),
                                         (lds_void *)(smem + sl * 4096 + wave * 1024), 16, 0, 0);
    bf16x8 ah[2], al[2], bh[8], bl[8];
    Bwd1Ctx<KA> c{smem, smem + BBUF, smem + BBUF, Q > 1 ? (unsigned)BBUF : 0u, smem + BBUF, 0u, gb, Q * BBUF,
                  g, ah, al, bh, bl, acc, h, j, (unsigned)lane * 16u, wave * 1024};
    if (Q > 1) {
        bwd1_copy_slice<0, X3 ? 16 : 8, false>(c);
        bwd1_copy_slice<1, X3 ? 16 : 8, false>(c);
    }
    if (h == 0) bwd1_gen_all<KA, true>(c, std::make_integer_sequence<int, 48>{});
    else bwd1_gen_all<KA, false>(c, std::make_integer_sequence<int, 48>{});
    // the lo halves of pair 3 (in the loop: slots 2 and 5 of the next step)
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        g[a].template half_lo<3>();
        ah[a] = g[a].hi();
        al[a] = g[a].lo();
    }
    wait_copies();
    __syncthreads();
#pragma unroll
    for (int b = 0; b < 8; ++b) bh[b] = bwd1_readb(smem, 0, b, 0, h, j);
    counted_lds_wait();   // known complete, these reads need no wait at the top of the loop

    for (int q = 0; q < Q; ++q) {
        c.cur = smem + (q & 1) * BBUF;
        c.nxt = smem + ((q & 1) ^ 1) * BBUF;
        c.cpy_dst = smem + (q & 1) * BBUF;
        c.cpy_off = (unsigned)min(q + 2, Q - 1) * (unsigned)BBUF;
        c.cpy_dst2 = smem + ((q & 1) ^ 1) * BBUF;
        c.cpy_off2 = (unsigned)min(q + 1, Q - 1) * (unsigned)BBUF;
        bwd1_slots<X3>(c, std::make_integer_sequence<int, X3 ? 192 : 64>{});
    }
    wait_copies();   // the copies issued in the last chunks must land before the buffers are reused
    __syncthreads();

    // Epilogue: g_i = sum_nn E_i,nn G[i][nn].  The accumulators hold G for rows
    // 32 a + 8 (r / 4) + 4 h + r % 4 of the wave and column n0 + 32 b + j; one column tile at a
    // time is transposed through LDS (rows of 36 floats: the b128 row reads of 16 lanes cover all
    // banks), after which lane l holds row l and walks its 32 columns with the epilogue recurrences.
    constexpr int EPS = 36;
    float *tb = (float *)smem + wave * (64 * EPS);
    const int64_t ibr = i0 + lane;
    const bool rvalid = ibr < n;
    EGen<E1, E2> eg;
    if (rvalid) eg.init(ax.te[ibr], n0, ax.pil);
    else eg.init(PhaseRec{}, n0, ax.pil);
    // Each 32-column run is summed in FP32, the runs of the tile in FP64.
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
        if (b == 0) g00 = gv[0];
        eg.seed();
        float nnp = (float)(n0 + 32 * b) * eg.pil;   // nn pi / L for the w sin kind
        float run = 0.0f, run2 = 0.0f;
#pragma unroll
        for (int k = 0; k < 32; ++k) {
            if constexpr (E1 == RUN_COSDIFF || E1 == RUN_SINDIFF) {
                run = fmaf(eg.c0.f * eg.c1.f, gv[k], run);
            } else if constexpr (E1 == RUN_COS) {
                run = fmaf(eg.c0.f, gv[k], run);
            } else {   // RUN_WSIN
                run = fmaf(nnp * eg.c0.f, gv[k], run);
            }
            if constexpr (EGen<E1, E2>::DUAL) run2 = fmaf(nnp * eg.c1.f, gv[k], run2);   // w sin of alpha
            if constexpr (E1 == RUN_WSIN || EGen<E1, E2>::DUAL) nnp += eg.pil;
            eg.c0.next();
            if constexpr (EGen<E1, E2>::HAS_C1) eg.c1.next();
        }
        sum += (double)run;
        if constexpr (EGen<E1, E2>::DUAL) sum2 += (double)run2;
        eg.rotate();
    }
    // kind factors: -2 sin sin (cosine differences), 2 cos sin (sine differences, nn = 0: the size)
    if constexpr (E1 == RUN_COSDIFF) sum *= -2.0;
    if constexpr (E1 == RUN_SINDIFF) {
        sum *= 2.0;
        if (n0 == 0) sum += (double)eg.size * (double)g00;   // 2 cos sin vanishes at nn = 0
    }
    if (rvalid) {
        ax.gpart[(size_t)ntile * (size_t)n + (size_t)ibr] = sum;
        if constexpr (EGen<E1, E2>::DUAL) ax.gpart2[(size_t)ntile * (size_t)n + (size_t)ibr] = sum2;
    }
}

// Row-form operand preparation for the bf16 path: BT[nn][k] = a_up times the factor of the form
// (gradient: 1 / scale of the K axis; potentials: 1 / (wt_u vt_p); point field: 1),
// split into bf16 hi and lo, zero padded, and tiled exactly in the LDS byte order of the gradient
// contractions (k_bwd1_bf16, k_bwd_bf16_st):
// tile (n_tile, q) = [hi | lo][256 rows][8 segments of 8 values], the 16-byte segment of logical
// index seg stored at seg ^ ((row / 2) % 8); logical segment seg = 4 half + s holds
// k = half * Kh + 32 q + 8 s + e (e = 0..7).
// trans = 0: nn = u, k = p (gx operand, a_up / vt_p);  trans = 1: nn = p, k = u (gy, a_up / wt_u).
__global__ void k_prep_bwd_bf16(int form, const double *__restrict__ a, int Mu, int Mp, double W, double H,
                                int trans, int Np, int Kh, unsigned short *__restrict__ B) {
    const int Q = Kh / 32;
    const size_t per_tile = (size_t)BBUF / 2;
    const size_t total = (size_t)(Np / BTN) * (size_t)Q * per_tile;
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= total) return;
    const size_t tile = idx / per_tile;
    const int within = (int)(idx % per_tile);
    const int hl = within / (BARR / 2);
    const int r = within % (BARR / 2);
    const int row = r / BKC, pseg = (r % BKC) / 8, e = r % 8;
    const int seg = pseg ^ ((row >> 1) & 7);
    const int half = seg >> 2, st = seg & 3;
    const int nt = (int)(tile / Q), q = (int)(tile % Q);
    const int nn = nt * BTN + row;
    const int k = half * Kh + 32 * q + 8 * st + e;
    const int Nb = trans ? Mp : Mu, Ka = trans ? Mu : Mp;
    float out = 0.0f;
    if (nn < Nb && k < Ka) {
        const int u = trans ? k : nn, p = trans ? nn : k;
        const double wt = u ? (double)u * kPi / W : 1.0, vt = p ? (double)p * kPi / H : 1.0;
        double sc = 1.0;                                  // ROW_POINT_*: a itself
        if (form == ROW_FIELD) sc = trans ? wt : vt;      // a / (scale of the K axis)
        else if (form == ROW_POTENTIAL) sc = wt * vt;     // a / (wt_u vt_p)
        const double v = a[(size_t)u * Mp + p] / sc;
        const float hv = (float)(__bf16)(float)v;
        out = hl == 0 ? hv : (float)(__bf16)(float)(v - (double)hv);
    }
    B[idx] = __builtin_bit_cast(unsigned short, (__bf16)out);
}

// ================================================================================================
// Store mode: the basis S_iu of one axis held in HBM as two bf16 tables (hi, lo), row-major
// [row = block][frequency], ld = frequencies rounded up to 256, rows = blocks rounded up to 256
// (rows past n are zero).  Built once per call from the phase records; the forward stages
// 32-block x 256-frequency tiles of both tables into LDS by direct global->LDS copies in exactly
// the swizzled byte order that the generating forward writes, and the backward loads its
// K-axis operand straight from the rows.
// ================================================================================================
template <bool X3>
__global__ __launch_bounds__(256) void k_build_table(int64_t n, int64_t nrows, int ld,
                                                     const PhaseRec *__restrict__ tab,
                                                     const RunSeed *__restrict__ seeds,
                                                     unsigned short *__restrict__ th,
                                                     unsigned short *__restrict__ tl) {
    const int runs = ld >> 5;
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= nrows * runs) return;
    const int64_t ib = idx / runs;
    const int r = (int)(idx % runs);
    const GenRec R = load_gen_at(tab, seeds, phase_rows(n), r, n, ib);
    float v[32];
    gen32(R, 32 * r, v);
    unsigned short *dh = th + (size_t)ib * (size_t)ld + 32 * r;
    unsigned short *dl = X3 ? tl + (size_t)ib * (size_t)ld + 32 * r : nullptr;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        unsigned hh[4], ll[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            if (X3) split2(v[8 * m + 2 * e], v[8 * m + 2 * e + 1], hh[e], ll[e]);
            else hh[e] = pack_bf16(v[8 * m + 2 * e], v[8 * m + 2 * e + 1]);
        }
        *(u32x4 *)(dh + 8 * m) = u32x4{hh[0], hh[1], hh[2], hh[3]};
        if (X3) *(u32x4 *)(dl + 8 * m) = u32x4{ll[0], ll[1], ll[2], ll[3]};
    }
}

// Direct copies of one chunk's four LDS tiles (Xh, Xl, Yh, Yl of 32 blocks x 256 frequencies):
// LDS byte o of a tile holds row k = o / 512, physical segment o / 16 % 32, i.e. logical segment
// (o / 16 % 32) ^ M(k) of the same row (the swizzle of fswz is an involution).
template <bool X3>
__device__ __forceinline__ void fwd_copy(const StoreTables &t, int64_t c, int tu0, int tp0, char *buf, int tid) {
    typedef __attribute__((address_space(3))) void lds_void;
    const int wave = tid >> 6, lane = tid & 63;
#pragma unroll
    for (int m = 0; m < 2; ++m) {
        const int o = m * 8192 + wave * 1024 + lane * 16;
        const int k = o >> 9, ps = (o >> 4) & 31;
        const int col = (ps ^ fswz_mask(k)) * 8;
        const size_t row = (size_t)(c * FKB + k);
        char *dst = buf + m * 8192 + wave * 1024;
        __builtin_amdgcn_global_load_lds((const void *)(t.xh + row * t.ldx + tu0 + col), (lds_void *)dst, 16, 0, 0);
        __builtin_amdgcn_global_load_lds((const void *)(t.yh + row * t.ldy + tp0 + col), (lds_void *)(dst + 2 * FARR),
                                         16, 0, 0);
        if (X3) {
            __builtin_amdgcn_global_load_lds((const void *)(t.xl + row * t.ldx + tu0 + col), (lds_void *)(dst + FARR),
                                             16, 0, 0);
            __builtin_amdgcn_global_load_lds((const void *)(t.yl + row * t.ldy + tp0 + col),
                                             (lds_void *)(dst + 3 * FARR), 16, 0, 0);
        }
    }
}

// Forward from stored tables: all 8 waves contract the current chunk while the next one streams
// into the other LDS buffer.  One-dimensional grid: the tiles of one K split go to the same XCD,
// where they run at about the same time and share its L2 copy of the split's table rows.
template <bool X3>
__global__ __launch_bounds__(512) void k_fwd_bf16_st(int Mu, int Mp, StoreTables t, float *__restrict__ part,
                                                     int tiles_u, int tiles_p, int splits, int64_t chunks,
                                                     int64_t chunks_per_split) {
    __shared__ __attribute__((aligned(16))) char smem[2 * FBUF];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int tiles = tiles_u * tiles_p;
    const int w = blockIdx.x, xcd = w & 7, slot = w >> 3;
    const int split = xcd + 8 * (slot / tiles), tile = slot % tiles;
    if (split >= splits) return;
    const int tu0 = (tile / tiles_p) * FT, tp0 = (tile % tiles_p) * FT;
    const int wu = 128 * (wave >> 2), wp = 64 * (wave & 3);
    const int64_t c_begin = (int64_t)split * chunks_per_split;
    const int64_t c_end = min(chunks, c_begin + chunks_per_split);

    f32x16 acc[4][2];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[a][b][r] = 0.0f;
    OpBase ox, oy;
    ox.init(wu, lane);
    oy.init(wp, lane);

    if (c_begin < c_end) {
        fwd_copy<X3>(t, c_begin, tu0, tp0, smem, tid);
        wait_copies();
    }
    __syncthreads();
    for (int64_t c = c_begin; c < c_end; ++c) {
        const int bsel = (int)((c - c_begin) & 1);
        char *cur = smem + bsel * FBUF, *nxt = smem + (bsel ^ 1) * FBUF;
        if (c + 1 < c_end) fwd_copy<X3>(t, c + 1, tu0, tp0, nxt, tid);
        fwd_mma<X3>(cur, ox, oy, acc);
        wait_copies();
        __syncthreads();
    }

    float *out = part + (size_t)split * (size_t)Mu * (size_t)Mp;
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

}  // namespace

hipError_t launch_phase_tables(int64_t n, const double *x, const double *y, const double *w, const double *h,
                               double W, double H, PhaseRec *tx, PhaseRec *ty, hipStream_t s) {
    if (n == 0) return hipSuccess;
    const int64_t rows = phase_rows(n);
    const unsigned g = (unsigned)((rows + 255) / 256);
    hipLaunchKernelGGL(k_phase_table, dim3(g), dim3(256), 0, s, n, rows, x, w, W, tx);
    hipLaunchKernelGGL(k_phase_table, dim3(g), dim3(256), 0, s, n, rows, y, h, H, ty);
    return hipGetLastError();
}

hipError_t launch_seed_table(int64_t n, int runs, const PhaseRec *tab, RunSeed *seeds, hipStream_t s) {
    if (n == 0) return hipSuccess;
    const int64_t rows = phase_rows(n);
    hipLaunchKernelGGL(k_seed_table, dim3((unsigned)((rows + 255) / 256)), dim3(256), 0, s, n, rows, runs, tab, seeds);
    return hipGetLastError();
}

hipError_t launch_fwd_bf16(const FwdPlan &pl, bool x3, int64_t n, int Mu, int Mp, const PhaseRec *tx,
                           const PhaseRec *ty, const RunSeed *sx, const RunSeed *sy, float *part, hipStream_t s) {
    if (pl.tu != FT || pl.tp != FT || pl.kb != FKB) return hipErrorInvalidValue;
    dim3 grid(pl.tiles_u * pl.tiles_p, pl.splits);
    if (x3)
        hipLaunchKernelGGL(k_fwd1_bf16<true>, grid, dim3(256), 0, s, n, Mu, Mp, tx, ty, sx, sy, part, pl.tiles_p,
                           pl.chunks, pl.chunks_per_split, 0, 0);
    else
        hipLaunchKernelGGL(k_fwd1_bf16<false>, grid, dim3(256), 0, s, n, Mu, Mp, tx, ty, sx, sy, part, pl.tiles_p,
                           pl.chunks, pl.chunks_per_split, 0, 0);
    return hipGetLastError();
}

hipError_t launch_fwd_bf16_mix(const FwdPlan &pl, int rx, int ry, int64_t n, int Mu, int Mp, const PhaseRec *tx,
                               const PhaseRec *ty, const RunSeed *sx, const RunSeed *sy, float *part, hipStream_t s) {
    if (pl.tu != FT || pl.tp != FT || pl.kb != FKB) return hipErrorInvalidValue;
    if (rx < 1 || ry < 1 || rx > pl.tiles_u || ry > pl.tiles_p) return hipErrorInvalidValue;
    // the rx x ry low-frequency tiles with three products (a grid over that corner alone: tiles_p = ry
    // maps its tile index to the same (u, p) tile), then every other tile with one; both write the
    // same split-K partials, so the reduction is unchanged
    hipLaunchKernelGGL(k_fwd1_bf16<true>, dim3(rx * ry, pl.splits), dim3(256), 0, s, n, Mu, Mp, tx, ty, sx, sy, part,
                       ry, pl.chunks, pl.chunks_per_split, 0, 0);
    if (rx < pl.tiles_u || ry < pl.tiles_p)
        hipLaunchKernelGGL(k_fwd1_bf16<false>, dim3(pl.tiles_u * pl.tiles_p, pl.splits), dim3(256), 0, s, n, Mu, Mp, tx,
                           ty, sx, sy, part, pl.tiles_p, pl.chunks, pl.chunks_per_split, rx, ry);
    return hipGetLastError();
}

hipError_t launch_prep_bwd_bf16(RowForm f, const double *a, int Mu, int Mp, double W, double H, int trans, int Np,
                                int Kh, unsigned short *B, hipStream_t s) {
    const size_t total = bwd_bf16_operand_elems(Np, Kh);
    hipLaunchKernelGGL(k_prep_bwd_bf16, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, (int)f, a, Mu, Mp, W,
                       H, trans, Np, Kh, B);
    return hipGetLastError();
}

size_t bwd_bf16_operand_elems(int Np, int Kh) { return (size_t)(Np / BTN) * (size_t)(Kh / 32) * (size_t)(BBUF / 2); }

namespace {
template <int KA, int E1, int E2>
hipError_t launch_rowform_bf16(bool x3, int64_t n, const BwdAxisBf16 &ax, hipStream_t s) {
    const int tiles_n = (ax.Nb + BTN - 1) / BTN;
    const int nt_end = ax.nt_end > 0 ? ax.nt_end : tiles_n;
    if (ax.nt0 < 0 || nt_end > tiles_n || ax.nt0 >= nt_end) return hipErrorInvalidValue;
    dim3 grid((unsigned)((n + 255) / 256), (unsigned)(nt_end - ax.nt0));
    if (x3) hipLaunchKernelGGL((k_bwd1_bf16<true, KA, E1, E2>), grid, dim3(256), 0, s, n, ax);
    else hipLaunchKernelGGL((k_bwd1_bf16<false, KA, E1, E2>), grid, dim3(256), 0, s, n, ax);
    return hipGetLastError();
}
}  // namespace

hipError_t launch_bwd_bf16(RowForm f, bool x3, int64_t n, const BwdAxisBf16 &ax, hipStream_t s) {
    if (n == 0) return hipSuccess;
    if (ax.tab_h) {
        // store mode (gradient only): one-dimensional XCD-aware grid over (block tile, N tile)
        if (f != ROW_FIELD || ax.tiles_b != (int)((n + 255) / 256) || ax.tiles_n != (ax.Nb + BTN - 1) / BTN ||
            ax.tab_ld < 2 * ax.Kh || (x3 && !ax.tab_l))
            return hipErrorInvalidValue;
        const unsigned g = (unsigned)((ax.tiles_b + 7) / 8 * 8 * ax.tiles_n);
        if (x3) hipLaunchKernelGGL(k_bwd_bf16_st<true>, dim3(g), dim3(512), 0, s, n, ax);
        else hipLaunchKernelGGL(k_bwd_bf16_st<false>, dim3(g), dim3(512), 0, s, n, ax);
        return hipGetLastError();
    }
    switch (f) {
        case ROW_FIELD: return launch_rowform_bf16<RUN_SINDIFF, RUN_COSDIFF, -1>(x3, n, ax, s);
        case ROW_POTENTIAL: return launch_rowform_bf16<RUN_SINDIFF, RUN_SINDIFF, -1>(x3, n, ax, s);
        case ROW_POINT_DUAL:
            if (!ax.gpart2) return hipErrorInvalidValue;
            return launch_rowform_bf16<RUN_COS, RUN_COS, RUN_WSIN>(x3, n, ax, s);
        case ROW_POINT_WSIN: return launch_rowform_bf16<RUN_COS, RUN_WSIN, -1>(x3, n, ax, s);
    }
    return hipErrorInvalidValue;
}

int64_t store_rows(int64_t n) { return (n + 255) / 256 * 256; }
int store_ld(int M) { return (M + 255) / 256 * 256; }

hipError_t launch_build_table(bool x3, int64_t n, int M, const PhaseRec *tab, const RunSeed *seeds,
                              unsigned short *th, unsigned short *tl, hipStream_t s) {
    const int64_t rows = store_rows(n);
    const int ld = store_ld(M);
    const int64_t total = rows * (ld / 32);
    if (total == 0) return hipSuccess;
    const unsigned g = (unsigned)((total + 255) / 256);
    if (x3) hipLaunchKernelGGL(k_build_table<true>, dim3(g), dim3(256), 0, s, n, rows, ld, tab, seeds, th, tl);
    else hipLaunchKernelGGL(k_build_table<false>, dim3(g), dim3(256), 0, s, n, rows, ld, tab, seeds, th, tl);
    return hipGetLastError();
}

hipError_t launch_fwd_bf16_st(const FwdPlan &pl, bool x3, int64_t n, int Mu, int Mp, const StoreTables &t,
                              float *part, hipStream_t s) {
    if (pl.tu != FT || pl.tp != FT || pl.kb != FKB) return hipErrorInvalidValue;
    if (t.ldx != store_ld(Mu) || t.ldy != store_ld(Mp) || pl.chunks * FKB > store_rows(n)) return hipErrorInvalidValue;
    const int tiles = pl.tiles_u * pl.tiles_p;
    const unsigned g = (unsigned)(tiles * ((pl.splits + 7) / 8 * 8));
    if (x3)
        hipLaunchKernelGGL(k_fwd_bf16_st<true>, dim3(g), dim3(512), 0, s, Mu, Mp, t, part, pl.tiles_u, pl.tiles_p,
                           pl.splits, pl.chunks, pl.chunks_per_split);
    else
        hipLaunchKernelGGL(k_fwd_bf16_st<false>, dim3(g), dim3(512), 0, s, Mu, Mp, t, part, pl.tiles_u, pl.tiles_p,
                           pl.splits, pl.chunks, pl.chunks_per_split);
    return hipGetLastError();
}

}  // namespace pp
