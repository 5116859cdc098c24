/*
 * pplace.h -- C ABI of the MI355X (gfx950) library for the truncated analytical cosine-series
 * solution of Poisson's equation with Neumann boundary conditions, driven by the exact
 * rectangle-block density (arXiv 2307.12041, Sec. III-A).
 *
 * Problem (Sec. II-A): a placement region [0, W] x [0, H] holding n rectangular blocks; block i
 * has centre (x_i, y_i) and size (w_i, h_i).  Its density is the sum of the block indicators
 * minus their mean (Sec. III-A, exact density and its mean-subtracted redefinition).
 *
 * Series (Sec. III-A, eq. psi): psi(x, y) = sum_{u<Mu} sum_{p<Mp} a_up cos(w_u x) cos(v_p y),
 * with w_u = u pi / W and v_p = p pi / H, truncated to u in [0, Mu), p in [0, Mp).
 *
 * Coefficients (Sec. III-A, the closed forms for a_{mu,eta}, a_{mu,0}, a_{0,eta}, and
 * a_00 = 0 from the compatibility condition): with the block integrals
 *     X_iu = integral of cos(w_u t) over [x_i - w_i/2, x_i + w_i/2]   (X_i0 = w_i),
 *     Y_ip = the same in y                                           (Y_i0 = h_i),
 * and the moments A_up = sum_i X_iu Y_ip,
 *     a_up = s_up A_up,   s_up = e_u e_p / (W H (w_u^2 + v_p^2)),  e_0 = 1, e_k = 2,  s_00 = 0.
 *
 * Energy (Sec. II-B, N = 1/2 sum_i q_i psi_i, read with the exact block density, so each block
 * contributes its charge density times psi integrated over its area):
 *     E = 1/2 iint rho psi = 1/2 sum_up a_up A_up.
 *
 * Gradient ("forces"; the field of eq. ksi integrated over each block, with the sign of a
 * gradient):  gx_i = dE/dx_i = sum_up a_up (cos(w_u x_i^+) - cos(w_u x_i^-)) Y_ip,
 *             gy_i = dE/dy_i = sum_up a_up X_iu (cos(v_p y_i^+) - cos(v_p y_i^-)).
 * The force on block i is -(gx_i, gy_i).
 *
 * Conventions for every entry point
 *   - Every array argument is a DEVICE pointer (memory of the current HIP device), owned by the
 *     caller, contiguous, 8-byte aligned.  Coefficient arrays are row-major, a[u * Mp + p].
 *   - ws is caller-owned device scratch of at least pp_workspace_size() bytes, 256-byte
 *     aligned.  The library allocates no memory and keeps no state between calls; concurrent
 *     calls need separate workspaces.
 *   - stream is a hipStream_t (NULL: the default stream).  Calls only enqueue work and return;
 *     outputs are valid once the stream has reached that point.  No call synchronises the host.
 *   - Return value: PP_OK (0) or a negative pp_status.  Argument errors are detected on the host
 *     before anything is enqueued, and then no output is touched.  PP_ERR_DEVICE means a launch
 *     failed; outputs are then undefined.  Non-finite block data is not checked (NaN in, NaN out).
 *   - Blocks may overhang the region; the series then integrates the whole block extent (the
 *     overhang is folded back by the even reflection that the Neumann cosine basis implies).
 */
#ifndef PPLACE_H
#define PPLACE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum pp_status {
    PP_OK = 0,
    PP_ERR_ARG = -1,          /* NULL pointer, bad or too large size, non-finite or non-positive W/H,
                                 misalignment */
    PP_ERR_WORKSPACE = -2,    /* ws_bytes smaller than pp_workspace_size() */
    PP_ERR_UNSUPPORTED = -3,  /* precision / basis mode not implemented by the library */
    PP_ERR_DEVICE = -4,       /* a HIP launch or runtime call failed */
    PP_ERR_SCRATCH = -5       /* pp_energy_static: the problem needs more than PP_STATIC_SCRATCH_BYTES */
} pp_status;

/* Arithmetic of the basis tables and the three contractions.  Seeds of the basis recurrences are
 * always reduced in FP64; the final reductions (coefficients, energy) are FP64; the per-block
 * gradient sums add runs of 32 columns in FP32 (bf16 paths; every column in the FP64 path) and
 * the runs in FP64. */
typedef enum pp_precision {
    PP_FP64 = 0,    /* FP64 tables, FP64 MFMA */
    PP_FP32 = 1,    /* FP32 tables (FP64 values rounded once), FP32 MFMA, FP32 accumulation */
    PP_BF16 = 2,    /* BF16 tables, BF16 MFMA, FP32 accumulation */
    PP_BF16X3 = 3,  /* BF16 hi/lo split of FP32 tables: hi*hi + hi*lo + lo*hi, FP32 accumulation */
    PP_FP8 = 4,     /* OCP e4m3 operands with E8M0 scales (v_mfma_scale_f32_32x32x64_f8f6f4), FP32
                       accumulation: the generated basis carried as v * 2^7 (scale 2^-7), the block sizes
                       (u = 0 row, p = 0 column) scaled by the largest size of each 64-block chunk, the
                       gradient's coefficient operand scaled per column and 64-value chunk; the k = 0 term
                       of the gradient contraction added exactly in FP32.  Relative error ~3e-2. */
    PP_FP8X3 = 5,   /* e4m3 hi/lo split of the same operands: hi*hi + lo*hi + hi*lo; relative error ~1e-3
                       (3 mantissa bits per part).  FP8 and FP8X3 serve pp_coeffs, pp_energy,
                       pp_energy_static and pp_field in recompute mode; pp_point_field,
                       pp_block_potential and the stored basis give PP_ERR_UNSUPPORTED. */
    PP_BF16MIX = 6  /* mixed split: PP_BF16X3 (three products) on the low-frequency tiles, PP_BF16 (hi only,
                       one product) elsewhere.  Per axis the first ceil(M / 1024) tiles of 256
                       frequencies (at least one: the first quarter of the frequencies) are split: the
                       coefficient contraction uses three products on the tiles with u and p both in
                       that range, the gradient contraction of gx (gy) on the N tiles of u (p) in it,
                       with the whole K axis.  The coefficients fall off like 1 / (u^2 + p^2)
                       (Sec. III-A), so the errors of the one-product tiles are small against the
                       largest terms of the energy and the gradient, which keep the accuracy of
                       PP_BF16X3 on placement-like inputs; each coefficient of those tiles on its own
                       is only as accurate as PP_BF16 makes it (~3e-3).  Serves pp_coeffs, pp_energy,
                       pp_energy_static and pp_field in recompute mode; pp_point_field,
                       pp_block_potential and the stored basis give PP_ERR_UNSUPPORTED. */
} pp_precision;

/* Where the basis values (the sine-difference factors of the Sec. III-A closed forms) live.
 * PP_BASIS_RECOMPUTE: generated on chip inside every contraction tile, never stored.
 * PP_BASIS_STORE (PP_BF16 and PP_BF16X3 only; other precisions give PP_ERR_UNSUPPORTED):
 *   pp_coeffs / pp_energy build the n x Mu and n x Mp tables (bf16 hi and lo) in the workspace and
 *   contract them from HBM; pp_field then READS the tables that the last pp_coeffs / pp_energy call
 *   left in the same workspace, so in this mode the workspace doubles as reserve space: pp_field
 *   must get the same problem, the same blocks and the same, unmodified workspace.  The tables
 *   take 2 (x3: 4) bytes per block and frequency of each axis (rows rounded up to 256 blocks,
 *   frequencies to 256). */
typedef enum pp_basis_mode {
    PP_BASIS_RECOMPUTE = 0,
    PP_BASIS_STORE = 1
} pp_basis_mode;

/* Problem description (Sec. II-A: region and blocks; truncation of the series, Sec. III-B/C).
 * The limits keep every launch grid of the library below 2^32 work-items per dimension; a problem
 * beyond them is rejected with PP_ERR_ARG before anything is enqueued:
 *   0 <= n <= 2^31 - 512;  1 <= Mu, Mp <= 65536 and Mu * Mp <= 2^30;
 *   PP_BASIS_STORE also needs ceil(n / 256) * ceil(max(Mu, Mp) / 256) < 2^21 (the table build).
 * (Memory is the caller's: pp_workspace_size() may ask for more than a device holds.) */
typedef struct pp_problem {
    double W, H;         /* region [0, W] x [0, H]; finite, > 0 */
    int64_t n;           /* number of blocks */
    int32_t Mu, Mp;      /* frequencies u in [0, Mu), p in [0, Mp) */
    int32_t precision;   /* pp_precision */
    int32_t basis_mode;  /* pp_basis_mode */
} pp_problem;

/* Bytes of device workspace that pp_coeffs, pp_energy, pp_field, pp_point_field and
 * pp_block_potential need for problem P (one size serves all of them).  Host only: makes no HIP
 * call. */
int pp_workspace_size(const pp_problem *P, size_t *bytes);

/* Series coefficients a_up (Sec. III-A closed forms; a_00 = 0).
 * x, y, w, h: [n] FP64 block centres and sizes.  a: out [Mu * Mp] FP64. */
int pp_coeffs(const pp_problem *P, const double *x, const double *y, const double *w, const double *h,
              double *a, void *ws, size_t ws_bytes, void *stream);

/* Energy E = 1/2 sum_up a_up A_up (Sec. II-B energy under the exact density) and optionally the
 * coefficients.  E: out, one FP64 value in device memory.  a: out [Mu * Mp] FP64, or NULL. */
int pp_energy(const pp_problem *P, const double *x, const double *y, const double *w, const double *h,
              double *E, double *a, void *ws, size_t ws_bytes, void *stream);

/* Bytes of the device array that serves pp_energy_static as its workspace (128 MiB). */
#define PP_STATIC_SCRATCH_BYTES (128u << 20)

/* pp_energy for callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): the same computation, kernels and results as
 * pp_energy, with the workspace taken from an array of PP_STATIC_SCRATCH_BYTES that the library
 * holds on each device it runs on until the process ends, instead of a caller workspace.  The call
 * allocates nothing (no hipMalloc, no allocating library routine; the first call on a device only
 * looks up the array's address there) and records no timing events.
 * Arguments, outputs and errors as for pp_energy; P->basis_mode must be PP_BASIS_RECOMPUTE
 * (PP_ERR_UNSUPPORTED otherwise); a problem whose pp_workspace_size() exceeds
 * PP_STATIC_SCRATCH_BYTES gives PP_ERR_SCRATCH before anything is enqueued.
 * Every call on one device shares that device's array: calls that may overlap on a device (other
 * streams, other host threads) race and must be serialised by the caller. */
int pp_energy_static(const pp_problem *P, const double *x, const double *y, const double *w, const double *h,
                     double *E, double *a, void *stream);

/* Per-block energy gradient, scaled by an upstream derivative (Sec. III-A field, eq. ksi,
 * integrated over each block).
 * a: in [Mu * Mp] FP64, the coefficients of the same problem and blocks (from pp_coeffs or
 *    pp_energy).  dE: in, one FP64 value in device memory, or NULL for 1.
 * gx, gy: out [n] FP64, gx_i = dE * dE/dx_i, gy_i = dE * dE/dy_i. */
int pp_field(const pp_problem *P, const double *x, const double *y, const double *w, const double *h,
             const double *a, const double *dE, double *gx, double *gy, void *ws, size_t ws_bytes,
             void *stream);

/* Point values of the potential and the field at npts = P->n points (Sec. III-A, eq. psi and
 * eq. ksi; the force of a point charge, Sec. II-B): at (px[k], py[k]),
 *   psi[k] = sum_up a_up cos(w_u px) cos(v_p py),
 *   xix[k] = sum_up a_up w_u sin(w_u px) cos(v_p py)  (= -d psi / dx),
 *   xiy[k] = sum_up a_up v_p cos(w_u px) sin(v_p py)  (= -d psi / dy).
 * Evaluation points may be the block centres or any other points (a grid for a picture of psi).
 * px, py: in [npts] FP64 device arrays.  a: in [Mu * Mp] FP64 coefficients (pp_coeffs).
 * psi, xix, xiy: out [npts] FP64, each may be NULL (not computed).
 * P->precision: the operand type of the contractions (FP64, FP32, BF16 or BF16X3; FP64 sums per
 * point); P->basis_mode must be PP_BASIS_RECOMPUTE (store gives PP_ERR_UNSUPPORTED).
 * ws: at least pp_workspace_size(P) bytes, P->n = npts.
 * Errors as for pp_field. */
int pp_point_field(const pp_problem *P, const double *px, const double *py, const double *a, double *psi,
                   double *xix, double *xiy, void *ws, size_t ws_bytes, void *stream);

/* Potential energy of each block against the whole density (Sec. II-B, N_i with the exact block
 * density, so that E = 1/2 sum_i N_i): N_i = integral of psi over block i
 *   = sum_up a_up Xbar_iu Ybar_ip,  Xbar_iu the sine-difference integral of block i (w_i at u = 0).
 * x, y, w, h: in [n] FP64 blocks.  a: in [Mu * Mp] FP64 coefficients of the same problem.
 * N: out [n] FP64.  P->precision: FP64, FP32, BF16 or BF16X3; P->basis_mode must be
 * PP_BASIS_RECOMPUTE (store gives PP_ERR_UNSUPPORTED).
 * Errors as for pp_field. */
int pp_block_potential(const pp_problem *P, const double *x, const double *y, const double *w, const double *h,
                       const double *a, double *N, void *ws, size_t ws_bytes, void *stream);

/* ---------------------------------------------------------------------------------------------
 * Bin scheme (Sec. III-D), a comparison path for the direct sum above.  The region is cut into
 * m x m bins of size wb = W/m, hb = H/m, centres x_l = (l + 1/2) wb, y_j = (j + 1/2) hb.  All
 * arithmetic is FP64; bin arrays are row-major, P[l * m + j] (l: x bin, j: y bin).
 * --------------------------------------------------------------------------------------------- */
typedef struct pp_bin_problem {
    double W, H;         /* region [0, W] x [0, H]; finite, > 0 */
    int64_t n;           /* blocks (pp_bin_density), 0 <= n < 2^31 */
    int32_t m;           /* bins per axis, 1 <= m <= 16384 */
    int32_t Mu, Mp;      /* truncation u in [0, Mu), p in [0, Mp); 1 <= Mu, Mp <= m */
} pp_bin_problem;

/* Bytes of device workspace that the pp_bin_* calls need for B (one size serves all three).
 * Host only. */
int pp_bin_workspace_size(const pp_bin_problem *B, size_t *bytes);

/* Bin densities (Sec. III-D, the density of bin b_lj): P_lj = area of the blocks inside bin lj
 * divided by wb hb, taken as the exact overlap areas (the "local smoothness" of the text is not
 * specified and is not applied); block parts outside the region lie in no bin.
 * x, y, w, h: in [B->n] FP64 blocks.  P: out [m * m] FP64.  FP64 atomic sums: the last bits may
 * differ between runs. */
int pp_bin_density(const pp_bin_problem *B, const double *x, const double *y, const double *w, const double *h,
                   double *P, void *ws, size_t ws_bytes, void *stream);

/* Binned coefficients (Sec. III-D, eqs. disa-a..d): the coefficients of the density
 * sum_lj P_lj [bin lj] minus its mean (eq. rho-dis), for u < Mu, p < Mp:
 *   a_00 = 0,
 *   a_0p = 4 H^2 / (p^3 pi^3 m) sin(p pi/(2m)) sum_lj P_lj cos(p (j + 1/2) pi/m),
 *   a_u0 = 4 W^2 / (u^3 pi^3 m) sin(u pi/(2m)) sum_lj P_lj cos(u (l + 1/2) pi/m),
 *   a_up = 16 W^2 H^2 sin(u pi/(2m)) sin(p pi/(2m)) / (u p (u^2 H^2 + p^2 W^2) pi^4)
 *          * sum_lj P_lj cos(u (l + 1/2) pi/m) cos(p (j + 1/2) pi/m).
 * P: in [m * m] FP64 (pp_bin_density, or any bin densities).  a: out [Mu * Mp] FP64. */
int pp_bin_coeffs(const pp_bin_problem *B, const double *P, double *a, void *ws, size_t ws_bytes, void *stream);

/* Potential and field at the bin centres, truncated at the coefficient array (Sec. III-D,
 * eqs. dis-psi1 and dis-ksi):
 *   psi[l, j] = sum_up a_up cos(u (l + 1/2) pi/m) cos(p (j + 1/2) pi/m),
 *   xix[l, j] = sum_up (u pi/W) a_up sin(u (l + 1/2) pi/m) cos(p (j + 1/2) pi/m),
 *   xiy[l, j] = sum_up (p pi/H) a_up cos(u (l + 1/2) pi/m) sin(p (j + 1/2) pi/m).
 * a: in [Mu * Mp] FP64 (pp_bin_coeffs, or the direct-sum coefficients for comparison).
 * psi, xix, xiy: out [m * m] FP64, each may be NULL (not computed). */
int pp_bin_field(const pp_bin_problem *B, const double *a, double *psi, double *xix, double *xiy, void *ws,
                 size_t ws_bytes, void *stream);

/* Block values from the bin-centre values (Sec. III-D, the final step of the fast scheme, whose
 * weights the text leaves open): each block takes the integral over its area of the bin values
 * held constant on each bin, i.e. the overlap-area weighted sum over the bins it covers,
 *   N[i]  =  sum_lj |block i cap bin lj| psi[l, j],
 *   gx[i] = -sum_lj |block i cap bin lj| xix[l, j],   gy[i] = -sum_lj |block i cap bin lj| xiy[l, j],
 * the bin-scheme counterparts of pp_block_potential and of the gradient of pp_field.  Block parts
 * outside the region take no bin.
 * x, y, w, h: in [B->n] FP64 blocks.  psi, xix, xiy: in [m * m] FP64 (pp_bin_field).  N, gx, gy:
 * out [B->n] FP64, none aliasing an input.  Each (field, output) pair is both NULL (skipped) or
 * both given; a NULL in only one of a pair is PP_ERR_ARG.  With B->n = 0 nothing is read or
 * written and every pointer may be NULL.  Results do not depend on scheduling
 * (per-block sums in a fixed order; blocks over more than 16 bins are summed by one workgroup
 * with a fixed-order reduction). */
int pp_bin_interp(const pp_bin_problem *B, const double *x, const double *y, const double *w, const double *h,
                  const double *psi, const double *xix, const double *xiy, double *N, double *gx, double *gy,
                  void *ws, size_t ws_bytes, void *stream);

/* Static description of a status code. */
const char *pp_strerror(int status);

/* Measurement hooks (they do not change any result).
 * pp_timing_enable(1) makes every later library call record a pair of HIP events around each
 * kernel launch it enqueues, on the caller's stream; pp_timing_enable(0) stops recording.  Either
 * call first discards all earlier records and their events.
 * pp_timing_query(name, &ms, &count) waits for the recorded events of one stage and returns their
 * summed duration in milliseconds and the number of launches.  Stage names: "tables" (per-block
 * phase records), "seeds" (run seeds of the bf16 forward), "fwd" (coefficient contraction), "reduce" (split-K sum, scale, energy
 * partials), "energy" (final energy sum), "prep" (row-form operands), "bwd" (the two gradient
 * contractions, one record each), "final" (per-block partial sums), "build" (store-mode basis
 * tables), "point" (pp_point_field
 * contractions), "potential" (pp_block_potential contraction), "bin_density", "bin_coeffs",
 * "bin_field", "bin_interp" (the bin scheme, all launches of one call in one record).  Unknown names give count 0.
 * Returns PP_OK, PP_ERR_ARG for NULL arguments, PP_ERR_DEVICE if an event query fails.  Recording
 * is process wide and guarded by a lock; it is meant for benchmarks, not for production calls. */
int pp_timing_enable(int on);
int pp_timing_query(const char *name, double *total_ms, int *count);

/* Matrix-core calibration (a measurement hook; it computes nothing of the method).
 * pp_mfma_calibrate(workgroups, iters, out, stream) enqueues one kernel of `workgroups` workgroups of
 * 256 threads (four waves).  Every wave issues 16 * iters v_mfma_f32_32x32x16_bf16 instructions into
 * 16 accumulator tiles and nothing else in its loop, on bf16 operands drawn from a standard normal
 * distribution (a counter-based hash of workgroup, thread and register), and each thread writes the
 * sum of its accumulators to out[workgroup * 256 + thread].  One call executes
 * workgroups * 4 * 16 * iters * 32768 flops; timed with events on `stream` it gives the bf16 rate the
 * matrix cores sustain on such data with every CU loaded (use a multiple of the CU count), which the
 * power limit, through the clock, holds well below the datasheet peak.
 * out: caller-owned device buffer of workgroups * 256 floats.  Returns PP_ERR_ARG for workgroups < 1
 * or > 65535, iters < 1 or out NULL, PP_ERR_DEVICE if the launch fails, else PP_OK. */
int pp_mfma_calibrate(int workgroups, int iters, float *out, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* PPLACE_H */
