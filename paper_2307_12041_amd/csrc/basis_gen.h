// basis_gen.h -- device helpers shared by the generating contractions (bf16 and fp8 kernels):
// FP64-reduced seeds, the fp32 sin/cos(pi r) polynomial, the three-term recurrence with a hi/lo
// coefficient, and the epilogue generator of the row-form contractions.
//
// Basis in product form (no cancellation for narrow blocks): for a block of centre c and size sz
// on an axis of length L, alpha = pi c / L, beta = pi sz / (2L), and frequency k >= 1,
//     S_k = sin(k (alpha + beta)) - sin(k (alpha - beta)) = 2 cos(k alpha) sin(k beta),
//     K_k = cos(k (alpha + beta)) - cos(k (alpha - beta)) = -2 sin(k alpha) sin(k beta),
// with S_0 = sz, K_0 = 0 (the sine- and cosine-difference factors of the closed-form
// coefficients, Sec. III-A, and of the field, eq. ksi).
#pragma once

#include "common.h"

namespace pp {
namespace gen {

__device__ __forceinline__ double reduce_half_turns(double t) { return t - 2.0 * rint(0.5 * t); }

// sin(pi r), cos(pi r) for |r| <= 1 in fp32: quarter-turn reduction f = r - q/2, |f| <= 1/4, then
// odd/even polynomials in f^2 (coefficients fitted by csrc/fit_sincospi.py; max error < 9e-8).
__device__ __forceinline__ void sincospi_seed(float r, float &s, float &c) {
    const float q = rintf(2.0f * r);
    const float f = fmaf(-0.5f, q, r);
    const float x = f * f;
    const float sp = f * fmaf(x, fmaf(x, fmaf(x, -5.893013400e-01f, 2.549791082e+00f), -5.167708535e+00f),
                              3.141592649e+00f);
    const float cp = fmaf(x, fmaf(x, fmaf(x, fmaf(x, 2.314641957e-01f, -1.335062776e+00f), 4.058708069e+00f),
                                  -4.934802175e+00f), 1.0f);
    const int iq = (int)q;
    const bool sw = iq & 1;
    const float s0 = sw ? cp : sp, c0 = sw ? sp : cp;
    // quadrant signs: q = 0: (s, c); 1: (c, -s); 2: (-s, -c); 3 (= -1): (-c, s)
    const unsigned ns = ((unsigned)iq & 2u) << 30, nc = ((unsigned)(iq + 1) & 2u) << 30;
    s = __builtin_bit_cast(float, __builtin_bit_cast(unsigned, s0) ^ ns);
    c = __builtin_bit_cast(float, __builtin_bit_cast(unsigned, c0) ^ nc);
}

// cos/sin of pi*(k*t) for integer k, with the product reduced in FP64 to [-1, 1] half turns.
__device__ __forceinline__ void seed_phasor(int k, double t, float &c, float &s) {
    const float r = (float)reduce_half_turns((double)k * t);
    sincospi_seed(r, s, c);
}

// Three-term recurrence state for cos(k alpha) (or any sinusoid) with a hi/lo coefficient.
//   next():  f_{k+1} = (ch + cl) f_k - f_{k-1}, the coefficient carried to ~2^-48 (the epilogue
//            generator);
//   next1(): f_{k+1} = ch f_k - f_{k-1}, one FMA (the basis generators).  Every run starts from
//            exact seeds and takes at most 31 steps; an error d in the coefficient then adds
//            d sum_i f_i U_{j-1-i} to value j (U the Chebyshev polynomials of the second kind, the
//            recurrence's own Green's function, |U_m| <= m + 1), at most ~d j^2 / 2 relative to
//            the run's values: d <= 2^-24 of 2cos(theta) gives ~6e-5 at j = 31 in the worst case, no
//            more than the fp32 rounding of the steps themselves grows to (both measured by an fp32
//            emulation: a worst absolute error of 3.8e-5 for 2 sin(k beta) over runs of 32 with the
//            one-FMA step, 3.0e-5 with the hi/lo coefficient; for cos(k alpha) 3.3e-5 and 2.9e-5).
struct Cheb {
    float f, fm, ch, cl;  // f_k, f_{k-1}, 2cos(theta) = ch + cl
    __device__ __forceinline__ float next() {
        const float nx = fmaf(ch, f, fmaf(cl, f, -fm));
        fm = f;
        f = nx;
        return nx;
    }
    __device__ __forceinline__ float next1() {
        const float nx = fmaf(ch, f, -fm);
        fm = f;
        f = nx;
        return nx;
    }
};

// Epilogue generator of one row (block) along the N axis: the recurrences of the epilogue kinds
// (sines or cosines of nn alpha, sine of nn beta), reseeded every 32 columns from phasors that
// advance by the 32-frequency rotations of the phase record.
template <int E1, int E2>
struct EGen {
    static constexpr bool DUAL = E2 >= 0;
    // chain 0 (alpha): cosine for SINDIFF and COS, sine for COSDIFF and WSIN; chain 1: sine of
    // alpha for the dual COS + WSIN epilogue, else sine of beta (SINDIFF, COSDIFF)
    static constexpr bool C0_COS = E1 == RUN_SINDIFF || E1 == RUN_COS;
    static constexpr bool HAS_C1 = DUAL || E1 == RUN_SINDIFF || E1 == RUN_COSDIFF;
    static constexpr bool C1_BETA = !DUAL;
    Cheb c0, c1;
    float pac, pas, pbc, pbs;     // phasors of alpha and beta at the current 32-column start
    float ca1, sa1, cb1, sb1;     // cos, sin of alpha and beta (one-column step)
    float ja_c, ja_s, jb_c, jb_s; // 32-column rotations
    float size, pil;

    __device__ __forceinline__ void init(const PhaseRec &R, int nn0, float pil_) {
        seed_phasor(nn0, R.ta, pac, pas);
        seed_phasor(nn0, R.tb, pbc, pbs);
        ca1 = R.ca; sa1 = R.sa; cb1 = R.cb; sb1 = R.sb;
        ja_c = R.ca32; ja_s = R.sa32; jb_c = R.cb32; jb_s = R.sb32;
        c0.ch = R.c2ah; c0.cl = R.c2al;
        if constexpr (C1_BETA) { c1.ch = R.c2bh; c1.cl = R.c2bl; }
        else { c1.ch = R.c2ah; c1.cl = R.c2al; }
        size = R.size;
        pil = pil_;
    }
    // chain values at the current start column nn and nn - 1
    __device__ __forceinline__ void seed() {
        if constexpr (C0_COS) { c0.f = pac; c0.fm = pac * ca1 + pas * sa1; }
        else { c0.f = pas; c0.fm = pas * ca1 - pac * sa1; }
        if constexpr (HAS_C1) {
            if constexpr (C1_BETA) { c1.f = pbs; c1.fm = pbs * cb1 - pbc * sb1; }
            else { c1.f = pas; c1.fm = pas * ca1 - pac * sa1; }
        }
    }
    __device__ __forceinline__ void rotate() {
        const float t = pac * ja_c - pas * ja_s;
        pas = pas * ja_c + pac * ja_s;
        pac = t;
        if constexpr (C1_BETA && HAS_C1) {
            const float tb = pbc * jb_c - pbs * jb_s;
            pbs = pbs * jb_c + pbc * jb_s;
            pbc = tb;
        }
    }
};

}  // namespace gen
}  // namespace pp
