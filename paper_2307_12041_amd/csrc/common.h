// common.h -- internal declarations shared by the HIP translation units of libpplace.
//
// Notation (arXiv 2307.12041, Sec. III-A): region [0,W] x [0,H], frequencies w_u = u pi / W,
// v_p = p pi / H.  On the device the basis tables are carried WITHOUT their 1/w_u factor:
//     S_iu = sin(w_u x_i^+) - sin(w_u x_i^-)   (u >= 1),   S_i0 = w_i,
//     T_ip = sin(v_p y_i^+) - sin(v_p y_i^-)   (p >= 1),   T_i0 = h_i,
//     K_iu = cos(w_u x_i^+) - cos(w_u x_i^-)   (u >= 1),   K_i0 = 0,   (L_ip likewise in y)
// so that X_iu = S_iu / wt_u with wt_u = w_u (u >= 1), wt_0 = 1, and the same for Y with vt_p.
// The device contraction is At = S^T T; then A = At / (wt_u vt_p), a = s_up A and
// E = 1/2 sum a A, where s_up is the spectral scale of the coefficient closed forms.
// Backward: gx_i = sum_u K_iu sum_p T_ip (a_up / vt_p), gy_i = sum_p L_ip sum_u S_iu (a_up / wt_u).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pp {

constexpr double kPi = 3.14159265358979323846;

// Work decomposition shared by the host (workspace sizing) and the launchers.
struct FwdPlan {
    int tu, tp;          // output tile of one workgroup (frequencies u x p)
    int kb;              // blocks per K chunk
    int tiles_u, tiles_p;
    int splits;          // split-K count
    int64_t chunks;      // ceil(n / kb)
    int64_t chunks_per_split;
    size_t part_elem;    // bytes per partial element (8: FP64, 4: FP32)
};

struct BwdPlan {
    int tb, tn, kk;      // block tile, output-frequency tile, K chunk (frequencies)
    int64_t tiles_b;     // ceil(n / tb)
    int tiles_nx;        // ceil(Mu / tn)  (gx: N = u)
    int tiles_ny;        // ceil(Mp / tn)  (gy: N = p)
    size_t bmat_elem;    // bytes per element of the prepared backward operand matrices
};

// Arguments of one backward contraction (gx or gy), see common.h header comment.
struct BwdAxis {
    const double *ca, *sa;   // K-side basis: coordinates and sizes (y,h for gx; x,w for gy)
    double La;               // K-side region length (H for gx, W for gy)
    int Ka;                  // K-side frequency count (Mp for gx, Mu for gy)
    const double *cb, *sb;   // epilogue basis: coordinates and sizes (x,w for gx; y,h for gy)
    double Lb;               // epilogue region length
    int Nb;                  // epilogue frequency count (Mu for gx, Mp for gy)
    const void *B;           // prepared operand [Ka][Nb] (layout depends on precision)
    double *gpart;           // out: [tiles_n][n] partial row sums (first epilogue)
    double *gpart2;          // out: [tiles_n][n] partial row sums of the second epilogue, if any
};

// Kinds of per-block basis values along one axis (frequency k, w_k = k pi / L, block centre c,
// size sz):
//   RUN_SINDIFF  sin(w_k (c + sz/2)) - sin(w_k (c - sz/2)), and sz at k = 0 (the sine-difference
//                integral times w_k, Sec. III-A coefficient closed forms);
//   RUN_COSDIFF  cos(w_k (c + sz/2)) - cos(w_k (c - sz/2)), 0 at k = 0 (its derivative, the field of
//                eq. ksi integrated over the block);
//   RUN_COS      cos(w_k c)  (point value of the eq. psi basis);
//   RUN_WSIN     w_k sin(w_k c)  (point value of the eq. ksi basis).
enum RunKind { RUN_SINDIFF = 0, RUN_COSDIFF = 1, RUN_COS = 2, RUN_WSIN = 3 };

// Which row-form contraction (FP64 / FP32 and bf16 kernels): K-side basis / epilogue basis.
enum RowForm {
    ROW_FIELD = 0,       // sine differences / cosine differences: the energy gradient (eq. ksi over a block)
    ROW_POTENTIAL = 1,   // sine differences / sine differences: block potentials (integral of eq. psi)
    ROW_POINT_DUAL = 2,  // cos / cos and w sin: point psi and xi along the epilogue axis
    ROW_POINT_WSIN = 3   // cos / w sin: point xi along the epilogue axis alone
};

// Per-block phase record of one axis, built once per call (80 bytes): for centre c, size sz and
// axis length L, ta = c / L and tb = sz / (2L) are the phases of the centre and half size in half
// turns per unit frequency; (ca, sa) = (cos, sin)(pi ta), c2a = 2 cos(pi ta) = c2ah + c2al, the
// same for tb, the 32-frequency phasors (ca32, sa32) and (cb32, sb32), and the size itself.  The
// four recurrence coefficients share one aligned 16-byte group (one load for the generators).
struct __attribute__((aligned(16))) PhaseRec {
    double ta, tb;
    float ca, sa, cb, sb;
    float c2ah, c2al, c2bh, c2bl;
    float ca32, sa32, cb32, sb32;
    float size, pad0, pad1, pad2;
};
static_assert(sizeof(PhaseRec) == 80, "PhaseRec layout");

// Start values of one run of 32 basis frequencies u0 = 32 r .. 32 r + 31 of one block (16 bytes):
// the two recurrences of the product form S_u = cos(u alpha) * 2 sin(u beta) begin from
// cf = cos(u0 alpha), cfm = cos((u0 - 1) alpha), sf = 2 sin(u0 beta), sfm = 2 sin((u0 - 1) beta),
// computed in FP64 and rounded once.  Table layout [run][row] (rows = phase_rows(n), zero past n),
// so that the 32 blocks of a chunk read one run's seeds from one contiguous 512-byte span.
struct __attribute__((aligned(16))) RunSeed {
    float cf, cfm, sf, sfm;
};
static_assert(sizeof(RunSeed) == 16, "RunSeed layout");

// Runs of a seed table for M frequencies: whole 256-frequency tiles of 8 runs each.
inline int seed_runs(int M) { return (M + 255) / 256 * 8; }

// Rows of a phase-record table: n rounded up to whole chunks of 32 blocks, plus two more chunks, all
// past n zero (an absent block: every basis value vanishes).  The bf16x3 forward fetches the
// records of the chunk after next without a bounds test.
__host__ __device__ inline int64_t phase_rows(int64_t n) { return (n + 31) / 32 * 32 + 64; }

// The (output tile, block split) of a forward workgroup on a grid of (tiles, splits).  Workgroups
// go to the 8 XCDs round-robin by linear id; taking ids in XCD-major order gives each XCD a
// contiguous run of splits, so the workgroups that read one split's per-block records (every tile
// of it) share that XCD's L2 instead of fetching the records once per XCD.
__device__ inline void fwd_tile_split(int &tile, int64_t &split) {
    const unsigned g = gridDim.x * gridDim.y, l = blockIdx.y * gridDim.x + blockIdx.x;
    const unsigned id = (g % 8u == 0u) ? (l % 8u) * (g / 8u) + l / 8u : l;
    tile = (int)(id % gridDim.x);
    split = (int64_t)(id / gridDim.x);
}

// One backward contraction of the bf16 path (gx or gy).
struct BwdAxisBf16 {
    const PhaseRec *ta;          // K-axis records (basis generated along K)
    const PhaseRec *te;          // epilogue-axis records (cosine differences)
    int Ka, Nb, Kh;              // K frequencies, N frequencies, K half length (multiple of 32)
    const unsigned short *B;     // tiled operand (hi and lo bf16, see k_prep_bwd_bf16)
    double *gpart;               // out: [tiles_n][n]
    // Store mode (tab_h non-NULL): the K-axis basis read from its stored tables instead of
    // generated; tab_ld is their row length, tiles_b / tiles_n the grid of block / N tiles.
    const unsigned short *tab_h, *tab_l;
    int tab_ld, tiles_b, tiles_n;
    // Row forms other than the gradient: a second epilogue's partial sums, and pi / L of the
    // epilogue axis (for the w sin kind).
    double *gpart2;
    float pil;
    // Recompute mode: the launch covers N tiles nt0 .. nt_end - 1 (nt_end = 0: all N tiles), so that
    // the mixed split can contract some N tiles with three products and the rest with one.
    int nt0, nt_end;
};

// One gradient contraction of the fp8 paths (gx or gy): as BwdAxisBf16 without store mode; B is the
// prepared e4m3 operand (k_prep_bwd_fp8 layout), B0 its exact k = 0 row (one float per N column).
struct BwdAxisFp8 {
    const PhaseRec *ta;          // K-axis records
    const PhaseRec *te;          // epilogue-axis records
    int Ka, Nb, Kh;              // K frequencies, N frequencies, K half length (multiple of 32)
    const unsigned char *B;
    const float *B0;
    double *gpart;               // out: [tiles_n][n]
    double *gpart2;              // unused by the gradient (one epilogue)
    float pil;
};

// Store-mode basis tables of both axes (bf16 hi and lo, row-major [block][frequency]).
struct StoreTables {
    const unsigned short *xh, *xl, *yh, *yl;
    int ldx, ldy;
};

// Brackets one kernel launch with HIP events when event timing is on (timing.hip); a NULL name
// marks a launch that is never timed (no event is created for it).
class TimedLaunch {
  public:
    TimedLaunch(const char *name, hipStream_t s);
    ~TimedLaunch();
  private:
    const char *name_;
    hipStream_t s_;
    void *start_ = nullptr, *stop_ = nullptr;
    bool active_ = false;
};

// ---- launchers (each defined next to its kernels) ----
hipError_t launch_fwd_f64(const FwdPlan &pl, int64_t n, int Mu, int Mp, double W, double H,
                          const double *x, const double *y, const double *w, const double *h,
                          double *part, hipStream_t s);
hipError_t launch_rowform_f64(RowForm f, const BwdPlan &pl, int64_t n, const BwdAxis &ax, hipStream_t s);
// FP32 operands on v_mfma_f32_16x16x4f32 (basis generated in FP64, rounded when stored; FP32
// accumulation inside a tile, FP64 across tiles).
hipError_t launch_fwd_f32(const FwdPlan &pl, int64_t n, int Mu, int Mp, double W, double H,
                          const double *x, const double *y, const double *w, const double *h,
                          float *part, hipStream_t s);
hipError_t launch_rowform_f32(RowForm f, const BwdPlan &pl, int64_t n, const BwdAxis &ax, hipStream_t s);
// Phase records of both axes (w, h may be NULL for points: size 0).
hipError_t launch_phase_tables(int64_t n, const double *x, const double *y, const double *w, const double *h,
                               double W, double H, PhaseRec *tx, PhaseRec *ty, hipStream_t s);
// Run seeds of one axis from its phase records (runs = seed_runs(M)).
hipError_t launch_seed_table(int64_t n, int runs, const PhaseRec *tab, RunSeed *seeds, hipStream_t s);
hipError_t launch_fwd_bf16(const FwdPlan &pl, bool x3, int64_t n, int Mu, int Mp, const PhaseRec *tx,
                           const PhaseRec *ty, const RunSeed *sx, const RunSeed *sy, float *part, hipStream_t s);
// Mixed split: the rx x ry low-frequency tiles with k_fwd1_bf16 (three products), the others with
// the one-product kernel; same partials and plan as launch_fwd_bf16.
hipError_t launch_fwd_bf16_mix(const FwdPlan &pl, int rx, int ry, int64_t n, int Mu, int Mp, const PhaseRec *tx,
                               const PhaseRec *ty, const RunSeed *sx, const RunSeed *sy, float *part, hipStream_t s);
hipError_t launch_prep_bwd_bf16(RowForm f, const double *a, int Mu, int Mp, double W, double H, int trans, int Np,
                                int Kh, unsigned short *B, hipStream_t s);
size_t bwd_bf16_operand_elems(int Np, int Kh);   // bf16 elements of one tiled backward operand
hipError_t launch_bwd_bf16(RowForm f, bool x3, int64_t n, const BwdAxisBf16 &ax, hipStream_t s);
// Store mode: table rows (n rounded up to 256) and row length (M rounded up to 256); the table of
// one axis from its phase records (lo table only for x3); the forward from both axes' tables.
int64_t store_rows(int64_t n);
int store_ld(int M);
hipError_t launch_build_table(bool x3, int64_t n, int M, const PhaseRec *tab, const RunSeed *seeds,
                              unsigned short *th, unsigned short *tl, hipStream_t s);
hipError_t launch_fwd_bf16_st(const FwdPlan &pl, bool x3, int64_t n, int Mu, int Mp, const StoreTables &t,
                              float *part, hipStream_t s);

// FP8 operand types (e4m3 on the scaled f8f6f4 MFMA): the coefficient contraction (chunks of 64
// blocks, 256 x 256 tiles, FP32 partials), the prepared gradient operand (bytes of one axis's
// tiles: fp8_operand_bytes; B0: Np floats) and the gradient contraction (ROW_FIELD only).
hipError_t launch_fwd_fp8(const FwdPlan &pl, bool x3, int64_t n, int Mu, int Mp, const PhaseRec *tx,
                          const PhaseRec *ty, const RunSeed *sx, const RunSeed *sy, float *part, hipStream_t s);
size_t fp8_operand_bytes(int Np, int Kh);
hipError_t launch_prep_bwd_fp8(RowForm f, const double *a, int Mu, int Mp, double W, double H, int trans, int Np,
                               int Kh, unsigned char *B, float *B0, hipStream_t s);
hipError_t launch_bwd_fp8(RowForm f, bool x3, int64_t n, const BwdAxisFp8 &ax, hipStream_t s);

// Sum split-K partials (FP64 or FP32), scale, write a, per-block energy partials.
hipError_t launch_reduce_scale(const void *part, bool part_f32, int splits, int Mu, int Mp, double W,
                               double H, double *a, double *epart, int *nblocks_out, hipStream_t s);
hipError_t launch_energy_final(const double *epart, int nblocks, double *E, hipStream_t s);
int reduce_scale_blocks(int Mu, int Mp);

// Row-form operand preparation from FP64 a (wt_u = w_u for u >= 1 and 1 at u = 0, vt_p likewise):
//   ROW_FIELD:      BxT[p][u] = a_up / vt_p,          By[u][p] = a_up / wt_u;
//   ROW_POTENTIAL:  BxT[p][u] = a_up / (vt_p wt_u),   By unused (may be NULL);
//   ROW_POINT_*:    BxT[p][u] = a_up,                 By[u][p] = a_up.
// A NULL output is skipped.
hipError_t launch_prep_rowform_f64(RowForm f, const double *a, int Mu, int Mp, double W, double H, double *BxT,
                                   double *By, hipStream_t s);
hipError_t launch_prep_rowform_f32(RowForm f, const double *a, int Mu, int Mp, double W, double H, float *BxT,
                                   float *By, hipStream_t s);
// gx[i] = dE * sum_t gpart_x[t][i], gy likewise (dE NULL: 1; a NULL output is skipped).
hipError_t launch_bwd_final(const double *gpx, int tx, const double *gpy, int ty, int64_t n,
                            const double *dE, double *gx, double *gy, hipStream_t s);

}  // namespace pp
