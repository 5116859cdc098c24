// bins.hip -- the bin scheme of Sec. III-D as a comparison path for the direct sum: exact bin
// densities, the binned coefficients (eqs. disa-a..d), the potential and field at the bin
// centres (eqs. dis-psi1, dis-ksi) and the block values weighted from the bins, all in FP64.
//
// The two cosine transforms of the coefficients and the inverse transforms of the field are
// separable: with C_f(s) = cos(f (2s+1) pi / (2m)) and S_f(s) = sin(...),
//     a'_up = sum_l C_u(l) sum_j P_lj C_p(j),                        a_up = disa factor(u,p) a'_up,
//     psi_lj = sum_u C_u(l) R_uj,   R_uj = sum_p a_up C_p(j),
//     xi_x,lj = sum_u (u pi/W) S_u(l) R_uj,   xi_y,lj = sum_u C_u(l) Rs_uj,  Rs_uj = sum_p a_up (p pi/H) S_p(j).
// Each is one FP64 MFMA GEMM whose trigonometric operand is read from a table of cos and sin of
// k pi / (2m), k in [0, 4m), indexed by f (2s+1) mod 4m (exact integer reduction, so every entry
// carries only the table's one rounding).
#include <math.h>

#include "common.h"
#include "pplace.h"

namespace pp {
namespace {

typedef double f64x4 __attribute__((ext_vector_type(4)));

// ------------------------------------------------------------------------------------------------
// Densities.  One thread per block adds its overlap with each bin it covers (FP64 atomics); a
// block covering more than kSmallBins bins is appended to a list that whole workgroups process.
// ------------------------------------------------------------------------------------------------
constexpr int kSmallBins = 16;

struct BinGeom {
    double W, H, wb, hb, inv_area;
    int m;
};

// Bin range [l0, l1] x [j0, j1] that block (x0..x1, y0..y1) may overlap; empty if l0 > l1.
__device__ __forceinline__ void bin_range(const BinGeom &g, double x0, double x1, double y0, double y1, int &l0,
                                          int &l1, int &j0, int &j1) {
    l0 = max(0, (int)floor(x0 / g.wb));
    l1 = min(g.m - 1, (int)floor(x1 / g.wb));
    j0 = max(0, (int)floor(y0 / g.hb));
    j1 = min(g.m - 1, (int)floor(y1 / g.hb));
    if (x1 <= 0.0 || y1 <= 0.0 || x0 >= g.W || y0 >= g.H) l1 = l0 - 1;
}

__device__ __forceinline__ void bin_add(const BinGeom &g, double *P, double x0, double x1, double y0, double y1, int l,
                                        int j) {
    const double ox = fmin(x1, (l + 1) * g.wb) - fmax(x0, l * g.wb);
    const double oy = fmin(y1, (j + 1) * g.hb) - fmax(y0, j * g.hb);
    if (ox > 0.0 && oy > 0.0) atomicAdd(&P[(size_t)l * g.m + j], ox * oy * g.inv_area);
}

__global__ void k_fill(size_t count, double *p) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = 0.0;
}

__global__ void k_zero_count(int *c) {
    if (threadIdx.x == 0) *c = 0;
}

__global__ void k_bin_density(int64_t n, const double *__restrict__ x, const double *__restrict__ y,
                              const double *__restrict__ w, const double *__restrict__ h, BinGeom g,
                              double *__restrict__ P, int *__restrict__ big, int *__restrict__ nbig) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double x0 = x[i] - 0.5 * w[i], x1 = x[i] + 0.5 * w[i];
    const double y0 = y[i] - 0.5 * h[i], y1 = y[i] + 0.5 * h[i];
    int l0, l1, j0, j1;
    bin_range(g, x0, x1, y0, y1, l0, l1, j0, j1);
    if (l1 < l0 || j1 < j0) return;
    if ((int64_t)(l1 - l0 + 1) * (j1 - j0 + 1) > kSmallBins) {
        big[atomicAdd(nbig, 1)] = (int)i;
        return;
    }
    for (int l = l0; l <= l1; ++l)
        for (int j = j0; j <= j1; ++j) bin_add(g, P, x0, x1, y0, y1, l, j);
}

// Workgroups take the listed blocks in turn; the threads of a workgroup share a block's bins.
__global__ void k_bin_density_big(const double *__restrict__ x, const double *__restrict__ y,
                                  const double *__restrict__ w, const double *__restrict__ h, BinGeom g,
                                  double *__restrict__ P, const int *__restrict__ big, const int *__restrict__ nbig) {
    const int count = *nbig;
    for (int t = blockIdx.x; t < count; t += gridDim.x) {
        const int i = big[t];
        const double x0 = x[i] - 0.5 * w[i], x1 = x[i] + 0.5 * w[i];
        const double y0 = y[i] - 0.5 * h[i], y1 = y[i] + 0.5 * h[i];
        int l0, l1, j0, j1;
        bin_range(g, x0, x1, y0, y1, l0, l1, j0, j1);
        const int nj = j1 - j0 + 1;
        const int64_t nb = (int64_t)(l1 - l0 + 1) * nj;
        for (int64_t b = threadIdx.x; b < nb; b += blockDim.x)
            bin_add(g, P, x0, x1, y0, y1, l0 + (int)(b / nj), j0 + (int)(b % nj));
    }
}

// ------------------------------------------------------------------------------------------------
// Block values from bin values (the last step of the scheme): each block takes the overlap-area
// weighted sum of the bins it covers, out_k[i] = sign_k sum_lj |block i cap bin lj| v_k[l, j], for
// the fields k that are present (psi -> N with sign +1, xi_x -> gx and xi_y -> gy with sign -1).
// One thread per block sums a block of up to kSmallBins bins in a fixed order; larger blocks go to
// a list, and one workgroup per listed block sums its bins and reduces in LDS in a fixed order, so
// every result is independent of scheduling.
// ------------------------------------------------------------------------------------------------
struct InterpIO {
    const double *v[3];
    double *out[3];
};

__device__ __forceinline__ void interp_bin(const BinGeom &g, const InterpIO &io, double x0, double x1, double y0,
                                           double y1, int l, int j, double acc[3]) {
    const double ox = fmin(x1, (l + 1) * g.wb) - fmax(x0, l * g.wb);
    const double oy = fmin(y1, (j + 1) * g.hb) - fmax(y0, j * g.hb);
    if (ox > 0.0 && oy > 0.0) {
        const double area = ox * oy;
        const size_t b = (size_t)l * g.m + j;
#pragma unroll
        for (int k = 0; k < 3; ++k)
            if (io.v[k]) acc[k] = fma(area, io.v[k][b], acc[k]);
    }
}

__device__ __forceinline__ void interp_store(const InterpIO &io, int64_t i, const double acc[3]) {
    if (io.v[0]) io.out[0][i] = acc[0];
    if (io.v[1]) io.out[1][i] = -acc[1];
    if (io.v[2]) io.out[2][i] = -acc[2];
}

__global__ void k_bin_interp(int64_t n, const double *__restrict__ x, const double *__restrict__ y,
                             const double *__restrict__ w, const double *__restrict__ h, BinGeom g, InterpIO io,
                             int *__restrict__ big, int *__restrict__ nbig) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double x0 = x[i] - 0.5 * w[i], x1 = x[i] + 0.5 * w[i];
    const double y0 = y[i] - 0.5 * h[i], y1 = y[i] + 0.5 * h[i];
    int l0, l1, j0, j1;
    bin_range(g, x0, x1, y0, y1, l0, l1, j0, j1);
    double acc[3] = {0.0, 0.0, 0.0};
    if (l1 >= l0 && j1 >= j0) {
        if ((int64_t)(l1 - l0 + 1) * (j1 - j0 + 1) > kSmallBins) {
            big[atomicAdd(nbig, 1)] = (int)i;
            return;
        }
        for (int l = l0; l <= l1; ++l)
            for (int j = j0; j <= j1; ++j) interp_bin(g, io, x0, x1, y0, y1, l, j, acc);
    }
    interp_store(io, i, acc);
}

constexpr int kInterpThreads = 256;

__global__ __launch_bounds__(kInterpThreads) void k_bin_interp_big(const double *__restrict__ x,
                                                                   const double *__restrict__ y,
                                                                   const double *__restrict__ w,
                                                                   const double *__restrict__ h, BinGeom g,
                                                                   InterpIO io, const int *__restrict__ big,
                                                                   const int *__restrict__ nbig) {
    __shared__ double red[3][kInterpThreads];
    const int count = *nbig;
    for (int t = blockIdx.x; t < count; t += gridDim.x) {
        const int i = big[t];
        const double x0 = x[i] - 0.5 * w[i], x1 = x[i] + 0.5 * w[i];
        const double y0 = y[i] - 0.5 * h[i], y1 = y[i] + 0.5 * h[i];
        int l0, l1, j0, j1;
        bin_range(g, x0, x1, y0, y1, l0, l1, j0, j1);
        const int nj = j1 - j0 + 1;
        const int64_t nb = (int64_t)(l1 - l0 + 1) * nj;
        double acc[3] = {0.0, 0.0, 0.0};
        for (int64_t b = threadIdx.x; b < nb; b += kInterpThreads)
            interp_bin(g, io, x0, x1, y0, y1, l0 + (int)(b / nj), j0 + (int)(b % nj), acc);
#pragma unroll
        for (int k = 0; k < 3; ++k) red[k][threadIdx.x] = acc[k];
        __syncthreads();
        for (int half = kInterpThreads / 2; half > 0; half >>= 1) {
            if ((int)threadIdx.x < half)
#pragma unroll
                for (int k = 0; k < 3; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + half];
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            const double tot[3] = {red[0][0], red[1][0], red[2][0]};
            interp_store(io, i, tot);
        }
        __syncthreads();
    }
}

// cos and sin of k pi / (2m), k in [0, 4m): tab[k] and tab[4m + k].
__global__ void k_bin_trig(int m, double *__restrict__ tab) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= 4 * m) return;
    double s, c;
    sincospi((double)k / (2.0 * m), &s, &c);
    tab[k] = c;
    tab[4 * m + k] = s;
}

// ------------------------------------------------------------------------------------------------
// GEMM C[M x N] = A[M x K] B[K x N] on v_mfma_f64_16x16x4f64, one operand a dense row-major
// matrix and the other a trigonometric view read from the table.
// ------------------------------------------------------------------------------------------------
struct BinOp {
    const double *ptr;   // dense: element (r, c) at ptr[r * ld + c]
    int ld;
    int trig;            // 0: dense; 1: cos; 2: sin of f (2s+1) pi / (2m)
    int freq_is_row;     // trig: f = r, s = c (1) or f = c, s = r (0)
    double wscale;       // trig: value times f * wscale, unless 0
};

// The load of element (r, c) of an operand whose kind (dense or trigonometric) is known at compile
// time, split so that nothing waits for it before it is stored: v receives the raw load (from a
// valid address even outside the matrix), sc the factor it is to be multiplied by.
template <bool TRIG>
__device__ __forceinline__ void binop_issue(const BinOp &o, const double *__restrict__ tab, int m4, int r, int c,
                                            bool valid, double &v, double &sc) {
    if constexpr (!TRIG) {
        v = o.ptr[valid ? (size_t)r * o.ld + c : 0];
        sc = 1.0;
    } else {
        const int f = o.freq_is_row ? r : c, s = o.freq_is_row ? c : r;
        // f < m and 2s + 1 < 2m, so the product is below 2 m^2 <= 2^29: exact in 32-bit unsigned
        const unsigned q = valid ? ((unsigned)f * (unsigned)(2 * s + 1)) % (unsigned)m4 : 0u;
        v = tab[(o.trig - 1) * m4 + (int)q];
        sc = o.wscale != 0.0 ? (double)f * o.wscale : 1.0;
    }
}

// Epilogue factor of the binned coefficients (eqs. disa-a..d) for row u, column p.
__device__ __forceinline__ double disa_factor(int u, int p, double W, double H, int m) {
    const double pi = kPi;
    if (u == 0 && p == 0) return 0.0;
    if (u == 0) return 4.0 * H * H / ((double)p * p * p * pi * pi * pi * m) * sinpi(p / (2.0 * m));
    if (p == 0) return 4.0 * W * W / ((double)u * u * u * pi * pi * pi * m) * sinpi(u / (2.0 * m));
    return 16.0 * W * W * H * H / ((double)u * p * ((double)u * u * H * H + (double)p * p * W * W) * pi * pi * pi * pi) *
           sinpi(u / (2.0 * m)) * sinpi(p / (2.0 * m));
}

// 128 x 128 output tile per workgroup of 8 waves (2 x 4 sub-tiles of 64 x 32, eight 16 x 16
// accumulators each); K chunks of 32 in LDS, A as [i][k] with rows of KP = 34 doubles and B as
// [k][j] with rows of JP = 144 doubles.  With 64 banks of 4 bytes, the MFMA operand reads (16
// lanes along i or j, the next 16 lanes one k further) and the stores (consecutive threads along
// k for A, along j for B) are then free of bank conflicts.  The operands of chunk c + 1 are
// fetched into registers while the MFMAs of chunk c run, then stored between two barriers.
constexpr int GT = 128, GK = 32, KP = GK + 2, JP = GT + 16, GTHREADS = 512;

template <bool DISA, bool ATRIG>
__global__ __launch_bounds__(GTHREADS) void k_bin_gemm(int M, int N, int K, BinOp A, BinOp B,
                                                       const double *__restrict__ tab, int m4,
                                                       double *__restrict__ C, int ldc, double W, double H, int m) {
    __shared__ double As[GT * KP];   // [i][k]
    __shared__ double Bs[GK * JP];   // [k][j]
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int r0 = blockIdx.y * GT, c0 = blockIdx.x * GT;
    const int wr = (wave >> 2) * 64, wc = (wave & 3) * 32;
    f64x4 acc[4][2];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = f64x4{0.0, 0.0, 0.0, 0.0};

    // One operand is trigonometric (ATRIG: A, else B), the other dense.
    constexpr int PER = GT * GK / GTHREADS;
    double na[PER], nb[PER], sa[PER], sb[PER];
    bool oka[PER], okb[PER];
    auto fetch = [&](int k0) {
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int e = tid + GTHREADS * q;
            const int ia = e / GK, ka = e % GK;      // A element (r0 + ia, k0 + ka)
            const int kb = e / GT, jb = e % GT;      // B element (k0 + kb, c0 + jb)
            const int ra = r0 + ia, ca = k0 + ka, rb = k0 + kb, cb = c0 + jb;
            oka[q] = ra < M && ca < K;
            okb[q] = rb < K && cb < N;
            binop_issue<ATRIG>(A, tab, m4, ra, ca, oka[q], na[q], sa[q]);
            binop_issue<!ATRIG>(B, tab, m4, rb, cb, okb[q], nb[q], sb[q]);
        }
    };
    auto stash = [&]() {
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int e = tid + GTHREADS * q;
            As[(e / GK) * KP + e % GK] = oka[q] ? na[q] * sa[q] : 0.0;
            Bs[(e / GT) * JP + e % GT] = okb[q] ? nb[q] * sb[q] : 0.0;
        }
    };
    fetch(0);
    stash();
    __syncthreads();
    for (int k0 = 0; k0 < K; k0 += GK) {
        const bool more = k0 + GK < K;
        if (more) fetch(k0 + GK);
#pragma unroll
        for (int ks = 0; ks < GK / 4; ++ks) {
            const int kr = 4 * ks + (lane >> 4);
            double av[4], bv[2];
#pragma unroll
            for (int a = 0; a < 4; ++a) av[a] = As[(wr + 16 * a + (lane & 15)) * KP + kr];
#pragma unroll
            for (int b = 0; b < 2; ++b) bv[b] = Bs[kr * JP + wc + 16 * b + (lane & 15)];
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], acc[a][b], 0, 0, 0);
        }
        if (more) {
            __syncthreads();
            stash();
        }
        __syncthreads();
    }
    // D layout of v_mfma_f64_16x16x4f64: row 4 r + lane / 16, column lane % 16.
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = r0 + wr + 16 * a + 4 * r + (lane >> 4);
                const int col = c0 + wc + 16 * b + (lane & 15);
                if (row < M && col < N) {
                    double v = acc[a][b][r];
                    if (DISA) v *= disa_factor(row, col, W, H, m);
                    C[(size_t)row * ldc + col] = v;
                }
            }
}

hipError_t gemm(int M, int N, int K, const BinOp &A, const BinOp &B, const double *tab, int m, double *C, int ldc,
                bool disa, double W, double H, hipStream_t s) {
    if (M <= 0 || N <= 0) return hipSuccess;
    dim3 grid((unsigned)((N + GT - 1) / GT), (unsigned)((M + GT - 1) / GT));
    // every transform has exactly one trigonometric operand
    if ((A.trig != 0) == (B.trig != 0)) return hipErrorInvalidValue;
    if (disa && A.trig)
        hipLaunchKernelGGL((k_bin_gemm<true, true>), grid, dim3(GTHREADS), 0, s, M, N, K, A, B, tab, 4 * m, C, ldc, W,
                           H, m);
    else if (disa)
        hipLaunchKernelGGL((k_bin_gemm<true, false>), grid, dim3(GTHREADS), 0, s, M, N, K, A, B, tab, 4 * m, C, ldc,
                           W, H, m);
    else if (A.trig)
        hipLaunchKernelGGL((k_bin_gemm<false, true>), grid, dim3(GTHREADS), 0, s, M, N, K, A, B, tab, 4 * m, C, ldc,
                           W, H, m);
    else
        hipLaunchKernelGGL((k_bin_gemm<false, false>), grid, dim3(GTHREADS), 0, s, M, N, K, A, B, tab, 4 * m, C, ldc,
                           W, H, m);
    return hipGetLastError();
}

BinOp dense(const double *p, int ld) { return BinOp{p, ld, 0, 0, 0.0}; }
BinOp trig(int kind, bool freq_is_row, double wscale) { return BinOp{nullptr, 0, kind, freq_is_row ? 1 : 0, wscale}; }

// Workspace: trig table (8m doubles), transform temporaries, big-block list (n + 1 ints).
struct BinLayout {
    size_t tab, tmp, list, total;
};

size_t align256(size_t v) { return (v + 255) / 256 * 256; }

BinLayout bin_layout(const pp_bin_problem &B) {
    BinLayout L{};
    const size_t m = (size_t)B.m;
    const size_t t1 = m * (size_t)B.Mp, t2 = 2 * (size_t)B.Mu * m;
    L.tab = 0;
    L.tmp = align256(8 * m * sizeof(double));
    L.list = L.tmp + align256((t1 > t2 ? t1 : t2) * sizeof(double));
    L.total = L.list + align256(((size_t)(B.n > 0 ? B.n : 0) + 1) * sizeof(int));
    return L;
}

bool finite_pos(double v) { return isfinite(v) && v > 0.0; }
bool al8(const void *p) { return ((uintptr_t)p & 7u) == 0; }

int check_bin_problem(const pp_bin_problem *B) {
    if (!B) return PP_ERR_ARG;
    if (!finite_pos(B->W) || !finite_pos(B->H)) return PP_ERR_ARG;
    if (B->n < 0 || B->n > (int64_t)0x7fffffff) return PP_ERR_ARG;
    if (B->m < 1 || B->m > 16384) return PP_ERR_ARG;
    if (B->Mu < 1 || B->Mp < 1 || B->Mu > B->m || B->Mp > B->m) return PP_ERR_ARG;
    return PP_OK;
}

int check_ws(const pp_bin_problem *B, void *ws, size_t ws_bytes) {
    const BinLayout L = bin_layout(*B);
    if (ws_bytes < L.total) return PP_ERR_WORKSPACE;
    if (!ws || ((uintptr_t)ws & 255u)) return PP_ERR_ARG;
    return PP_OK;
}

hipError_t fill_trig(int m, double *tab, hipStream_t s) {
    hipLaunchKernelGGL(k_bin_trig, dim3((unsigned)((4 * m + 255) / 256)), dim3(256), 0, s, m, tab);
    return hipGetLastError();
}

}  // namespace
}  // namespace pp

using namespace pp;

extern "C" {

int pp_bin_workspace_size(const pp_bin_problem *B, size_t *bytes) {
    int st = check_bin_problem(B);
    if (st != PP_OK) return st;
    if (!bytes) return PP_ERR_ARG;
    *bytes = bin_layout(*B).total;
    return PP_OK;
}

int pp_bin_density(const pp_bin_problem *B, const double *x, const double *y, const double *w, const double *h,
                   double *P, void *ws, size_t ws_bytes, void *stream) {
    int st = check_bin_problem(B);
    if (st != PP_OK) return st;
    if (!P || !al8(P)) return PP_ERR_ARG;
    if (B->n > 0 && (!x || !y || !w || !h || !al8(x) || !al8(y) || !al8(w) || !al8(h))) return PP_ERR_ARG;
    if ((st = check_ws(B, ws, ws_bytes)) != PP_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    const BinLayout L = bin_layout(*B);
    int *list = (int *)((char *)ws + L.list);
    const size_t mm = (size_t)B->m * (size_t)B->m;
    BinGeom g{B->W, B->H, B->W / B->m, B->H / B->m, 1.0 / ((B->W / B->m) * (B->H / B->m)), B->m};
    {
        TimedLaunch t("bin_density", s);
        hipLaunchKernelGGL(k_fill, dim3((unsigned)((mm + 255) / 256)), dim3(256), 0, s, mm, P);
        hipLaunchKernelGGL(k_zero_count, dim3(1), dim3(64), 0, s, list);
        if (B->n > 0) {
            hipLaunchKernelGGL(k_bin_density, dim3((unsigned)((B->n + 255) / 256)), dim3(256), 0, s, B->n, x, y, w, h, g,
                               P, list + 1, list);
            hipLaunchKernelGGL(k_bin_density_big, dim3(1024), dim3(256), 0, s, x, y, w, h, g, P, list + 1, list);
        }
        if (hipGetLastError() != hipSuccess) return PP_ERR_DEVICE;
    }
    return PP_OK;
}

int pp_bin_coeffs(const pp_bin_problem *B, const double *P, double *a, void *ws, size_t ws_bytes, void *stream) {
    int st = check_bin_problem(B);
    if (st != PP_OK) return st;
    if (!P || !a || !al8(P) || !al8(a)) return PP_ERR_ARG;
    if ((st = check_ws(B, ws, ws_bytes)) != PP_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    const BinLayout L = bin_layout(*B);
    double *tab = (double *)((char *)ws + L.tab), *Q = (double *)((char *)ws + L.tmp);
    const int m = B->m;
    TimedLaunch t("bin_coeffs", s);
    if (fill_trig(m, tab, s) != hipSuccess) return PP_ERR_DEVICE;
    // Q[l][p] = sum_j P[l][j] C_p(j);  a[u][p] = disa(u,p) sum_l C_u(l) Q[l][p]
    if (gemm(m, B->Mp, m, dense(P, m), trig(1, false, 0.0), tab, m, Q, B->Mp, false, B->W, B->H, s) != hipSuccess)
        return PP_ERR_DEVICE;
    if (gemm(B->Mu, B->Mp, m, trig(1, true, 0.0), dense(Q, B->Mp), tab, m, a, B->Mp, true, B->W, B->H, s) !=
        hipSuccess)
        return PP_ERR_DEVICE;
    return PP_OK;
}

int pp_bin_field(const pp_bin_problem *B, const double *a, double *psi, double *xix, double *xiy, void *ws,
                 size_t ws_bytes, void *stream) {
    int st = check_bin_problem(B);
    if (st != PP_OK) return st;
    if (!a || !al8(a)) return PP_ERR_ARG;
    if ((psi && !al8(psi)) || (xix && !al8(xix)) || (xiy && !al8(xiy))) return PP_ERR_ARG;
    if ((st = check_ws(B, ws, ws_bytes)) != PP_OK) return st;
    if (!psi && !xix && !xiy) return PP_OK;
    hipStream_t s = (hipStream_t)stream;
    const BinLayout L = bin_layout(*B);
    const int m = B->m, Mu = B->Mu, Mp = B->Mp;
    double *tab = (double *)((char *)ws + L.tab);
    double *R = (double *)((char *)ws + L.tmp), *Rs = R + (size_t)Mu * m;
    const double wu = kPi / B->W, vp = kPi / B->H;
    TimedLaunch t("bin_field", s);
    if (fill_trig(m, tab, s) != hipSuccess) return PP_ERR_DEVICE;
    // R[u][j] = sum_p a[u][p] C_p(j);  Rs[u][j] = sum_p a[u][p] (p pi/H) S_p(j)
    if ((psi || xix) && gemm(Mu, m, Mp, dense(a, Mp), trig(1, true, 0.0), tab, m, R, m, false, B->W, B->H, s) != hipSuccess)
        return PP_ERR_DEVICE;
    if (xiy && gemm(Mu, m, Mp, dense(a, Mp), trig(2, true, vp), tab, m, Rs, m, false, B->W, B->H, s) != hipSuccess)
        return PP_ERR_DEVICE;
    // psi[l][j] = sum_u C_u(l) R[u][j];  xi_x = sum_u (u pi/W) S_u(l) R[u][j];  xi_y = sum_u C_u(l) Rs[u][j]
    if (psi && gemm(m, m, Mu, trig(1, false, 0.0), dense(R, m), tab, m, psi, m, false, B->W, B->H, s) != hipSuccess)
        return PP_ERR_DEVICE;
    if (xix && gemm(m, m, Mu, trig(2, false, wu), dense(R, m), tab, m, xix, m, false, B->W, B->H, s) != hipSuccess)
        return PP_ERR_DEVICE;
    if (xiy && gemm(m, m, Mu, trig(1, false, 0.0), dense(Rs, m), tab, m, xiy, m, false, B->W, B->H, s) != hipSuccess)
        return PP_ERR_DEVICE;
    return PP_OK;
}

int pp_bin_interp(const pp_bin_problem *B, const double *x, const double *y, const double *w, const double *h,
                  const double *psi, const double *xix, const double *xiy, double *N, double *gx, double *gy, void *ws,
                  size_t ws_bytes, void *stream) {
    int st = check_bin_problem(B);
    if (st != PP_OK) return st;
    if (B->n == 0) return PP_OK;   // nothing read or written
    if (!psi != !N || !xix != !gx || !xiy != !gy) return PP_ERR_ARG;
    const void *ptrs[6] = {psi, xix, xiy, N, gx, gy};
    for (const void *p : ptrs)
        if (p && !al8(p)) return PP_ERR_ARG;
    if (!x || !y || !w || !h || !al8(x) || !al8(y) || !al8(w) || !al8(h)) return PP_ERR_ARG;
    if ((st = check_ws(B, ws, ws_bytes)) != PP_OK) return st;
    if (!psi && !xix && !xiy) return PP_OK;
    hipStream_t s = (hipStream_t)stream;
    const BinLayout L = bin_layout(*B);
    int *list = (int *)((char *)ws + L.list);
    BinGeom g{B->W, B->H, B->W / B->m, B->H / B->m, 1.0 / ((B->W / B->m) * (B->H / B->m)), B->m};
    InterpIO io{{psi, xix, xiy}, {N, gx, gy}};
    TimedLaunch t("bin_interp", s);
    hipLaunchKernelGGL(k_zero_count, dim3(1), dim3(64), 0, s, list);
    hipLaunchKernelGGL(k_bin_interp, dim3((unsigned)((B->n + 255) / 256)), dim3(256), 0, s, B->n, x, y, w, h, g, io,
                       list + 1, list);
    hipLaunchKernelGGL(k_bin_interp_big, dim3(1024), dim3(kInterpThreads), 0, s, x, y, w, h, g, io, list + 1, list);
    if (hipGetLastError() != hipSuccess) return PP_ERR_DEVICE;
    return PP_OK;
}

}  // extern "C"
