// api.hip -- the C ABI of include/pplace.h: argument validation (host only, before any enqueue),
// work decomposition, workspace layout and the launch sequence of each entry point.
#include <math.h>
#include <string.h>

#include <mutex>

#include "../../include/pplace.h"
#include "common.h"

// Workspace of pp_energy_static, for callers that cannot allocate: one copy of this array on
// every device the library runs on, held until the process ends.  Host code never uses the name
// itself (on the host it is only a stand-in); it uses the device address that
// hipGetSymbolAddress gives once per device (scratch_on_current_device below).
static __device__ __align__(256) char scratch[PP_STATIC_SCRATCH_BYTES];

namespace pp {
namespace {

constexpr int kMaxFreq = 65536;
// Largest block count and frequency-pair count: every launch grid of the library then stays below
// 2^32 work-items per dimension (the gradient launches take ceil(n / 256) x 512 or ceil(n / 128) x 256
// work-items, the coefficient-side launches about 2 Mu Mp); grids_fit() checks each one exactly.
constexpr int64_t kMaxBlocks = ((int64_t)1 << 31) - 512;
constexpr int64_t kMaxPairs = (int64_t)1 << 30;
constexpr size_t kAlign = 256;

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

bool supported_precision(int prec) {
    return prec == PP_FP64 || prec == PP_FP32 || prec == PP_BF16 || prec == PP_BF16X3 || prec == PP_FP8 ||
           prec == PP_FP8X3 || prec == PP_BF16MIX;
}
bool is_bf16(int prec) { return prec == PP_BF16 || prec == PP_BF16X3 || prec == PP_BF16MIX; }

// Mixed split: the low-frequency tiles that take three products, per axis: ceil(M / 1024) tiles of
// 256 frequencies (at least one, at most all), i.e. the first quarter of the frequencies.
int mix_tiles(int M) {
    const int r = (M + 1023) / 1024, t = (M + 255) / 256;
    return r < 1 ? 1 : (r > t ? t : r);
}
bool is_fp8(int prec) { return prec == PP_FP8 || prec == PP_FP8X3; }
// Operand types whose basis is generated from per-block phase records and run seeds.
bool is_gen(int prec) { return is_bf16(prec) || is_fp8(prec); }

bool grids_fit(const pp_problem &P);

int validate_problem(const pp_problem *P) {
    if (!P) return PP_ERR_ARG;
    if (!(isfinite(P->W) && P->W > 0.0) || !(isfinite(P->H) && P->H > 0.0)) return PP_ERR_ARG;
    if (P->n < 0 || P->n > kMaxBlocks) return PP_ERR_ARG;
    if (P->Mu < 1 || P->Mp < 1 || P->Mu > kMaxFreq || P->Mp > kMaxFreq) return PP_ERR_ARG;
    if ((int64_t)P->Mu * (int64_t)P->Mp > kMaxPairs) return PP_ERR_ARG;
    if (P->precision < PP_FP64 || P->precision > PP_BF16MIX) return PP_ERR_ARG;
    if (P->basis_mode != PP_BASIS_RECOMPUTE && P->basis_mode != PP_BASIS_STORE) return PP_ERR_ARG;
    if (!supported_precision(P->precision)) return PP_ERR_UNSUPPORTED;
    if (P->basis_mode == PP_BASIS_STORE && (!is_bf16(P->precision) || P->precision == PP_BF16MIX))
        return PP_ERR_UNSUPPORTED;
    if (!grids_fit(*P)) return PP_ERR_ARG;
    return PP_OK;
}

bool aligned8(const void *p) { return ((uintptr_t)p & 7u) == 0; }

int validate_blocks(const pp_problem *P, const double *x, const double *y, const double *w, const double *h) {
    if (P->n == 0) return PP_OK;
    if (!x || !y || !w || !h) return PP_ERR_ARG;
    if (!aligned8(x) || !aligned8(y) || !aligned8(w) || !aligned8(h)) return PP_ERR_ARG;
    return PP_OK;
}

FwdPlan fwd_plan(const pp_problem &P) {
    FwdPlan pl{};
    if (is_bf16(P.precision)) {
        pl.tu = 256; pl.tp = 256; pl.kb = 32;
    } else if (is_fp8(P.precision)) {
        pl.tu = 256; pl.tp = 256; pl.kb = 64;
    } else if (P.Mu >= 128 && P.Mp >= 128) {
        pl.tu = 128; pl.tp = 128; pl.kb = 32;
    } else {
        pl.tu = 64; pl.tp = 64; pl.kb = 32;
    }
    pl.tiles_u = (P.Mu + pl.tu - 1) / pl.tu;
    pl.tiles_p = (P.Mp + pl.tp - 1) / pl.tp;
    pl.chunks = (P.n + pl.kb - 1) / pl.kb;
    const int64_t tiles = (int64_t)pl.tiles_u * pl.tiles_p;
    // Enough workgroups to fill 256 CUs several times over, never more splits than chunks.  The mixed
    // split runs its few three-product tiles in a launch of their own, which needs as many
    // workgroups: at least 512 there.
    const int64_t target = 2048;
    int64_t splits = (target + tiles - 1) / tiles;
    if (P.precision == PP_BF16MIX) {
        const int64_t corner = (int64_t)mix_tiles(P.Mu) * mix_tiles(P.Mp);
        const int64_t need = (512 + corner - 1) / corner;
        if (splits < need) splits = need;
    }
    if (splits > pl.chunks) splits = pl.chunks;
    if (splits > 4096) splits = 4096;
    if (splits < 1) splits = 1;
    pl.chunks_per_split = (pl.chunks + splits - 1) / splits;
    if (pl.chunks_per_split < 1) pl.chunks_per_split = 1;
    pl.splits = (int)((pl.chunks + pl.chunks_per_split - 1) / pl.chunks_per_split);
    if (pl.splits < 1) pl.splits = 1;
    pl.part_elem = P.precision == PP_FP64 ? 8 : 4;
    return pl;
}

BwdPlan bwd_plan(const pp_problem &P) {
    BwdPlan pl{};
    if (is_gen(P.precision)) {
        pl.tb = 256; pl.tn = 256; pl.kk = 32;
    } else {
        pl.tb = 128; pl.tn = 128; pl.kk = 32;
    }
    pl.tiles_b = (P.n + pl.tb - 1) / pl.tb;
    pl.tiles_nx = (P.Mu + pl.tn - 1) / pl.tn;
    pl.tiles_ny = (P.Mp + pl.tn - 1) / pl.tn;
    pl.bmat_elem = P.precision == PP_FP32 ? 4 : 8;
    return pl;
}

// K half length of the bf16 backward (K frequencies split over the two lane halves; chunks of 32
// per half).
int bf16_kh(int Ka) { return (Ka + 63) / 64 * 32; }

// Workspace layout.  The phase tables (bf16 path) sit at the start of both regions; the forward
// region (partials, energy partials) and the backward region (operands, gradient partials) overlap.
struct Layout {
    size_t tx, ty;                       // bf16 path: per-block phase records
    size_t sxh, sxl, syh, syl;           // store mode: basis tables (kept from the forward to the backward)
    size_t sdx, sdy;                     // bf16 forward: run seeds of both axes
    size_t part, epart;                  // forward region
    size_t bx, by, gpx, gpy, gpz;        // backward region (gpz: second epilogue of the point field)
    size_t b0x, b0y;                     // fp8 gradient: exact k = 0 rows of the operands
    size_t fwd_bytes, bwd_bytes, total;
};

Layout layout(const pp_problem &P) {
    const FwdPlan f = fwd_plan(P);
    const BwdPlan b = bwd_plan(P);
    const size_t MM = (size_t)P.Mu * (size_t)P.Mp;
    Layout L{};
    size_t off = 0;
    if (is_gen(P.precision)) {
        L.tx = off; off = align_up(off + (size_t)phase_rows(P.n) * sizeof(PhaseRec));
        L.ty = off; off = align_up(off + (size_t)phase_rows(P.n) * sizeof(PhaseRec));
    }
    if (P.basis_mode == PP_BASIS_STORE) {
        const bool x3 = P.precision == PP_BF16X3;
        const size_t rows = (size_t)store_rows(P.n);
        const size_t bx = rows * (size_t)store_ld(P.Mu) * 2, by = rows * (size_t)store_ld(P.Mp) * 2;
        L.sxh = off; off = align_up(off + bx);
        if (x3) { L.sxl = off; off = align_up(off + bx); }
        L.syh = off; off = align_up(off + by);
        if (x3) { L.syl = off; off = align_up(off + by); }
    }
    const size_t common = off;
    if (is_gen(P.precision)) {
        const size_t rows = (size_t)phase_rows(P.n);
        L.sdx = off; off = align_up(off + (size_t)seed_runs(P.Mu) * rows * sizeof(RunSeed));
        L.sdy = off; off = align_up(off + (size_t)seed_runs(P.Mp) * rows * sizeof(RunSeed));
    }
    L.part = off;  off = align_up(off + (size_t)f.splits * MM * f.part_elem);
    L.epart = off; off = align_up(off + (size_t)reduce_scale_blocks(P.Mu, P.Mp) * sizeof(double));
    L.fwd_bytes = off;
    off = common;
    if (is_bf16(P.precision)) {
        const size_t ex = bwd_bf16_operand_elems(b.tiles_nx * 256, bf16_kh(P.Mp)) * 2;  // gx operand, bytes
        const size_t ey = bwd_bf16_operand_elems(b.tiles_ny * 256, bf16_kh(P.Mu)) * 2;  // gy operand, bytes
        L.bx = off;  off = align_up(off + ex);
        L.by = off;  off = align_up(off + ey);
    } else if (is_fp8(P.precision)) {
        L.bx = off;  off = align_up(off + fp8_operand_bytes(b.tiles_nx * 256, bf16_kh(P.Mp)));
        L.by = off;  off = align_up(off + fp8_operand_bytes(b.tiles_ny * 256, bf16_kh(P.Mu)));
        L.b0x = off; off = align_up(off + (size_t)b.tiles_nx * 256 * sizeof(float));
        L.b0y = off; off = align_up(off + (size_t)b.tiles_ny * 256 * sizeof(float));
    } else {
        L.bx = off;  off = align_up(off + MM * b.bmat_elem);
        L.by = off;  off = align_up(off + MM * b.bmat_elem);
    }
    L.gpx = off; off = align_up(off + (size_t)b.tiles_nx * (size_t)P.n * sizeof(double));
    L.gpy = off; off = align_up(off + (size_t)b.tiles_ny * (size_t)P.n * sizeof(double));
    L.gpz = off; off = align_up(off + (size_t)b.tiles_nx * (size_t)P.n * sizeof(double));
    L.bwd_bytes = off;
    L.total = L.fwd_bytes > L.bwd_bytes ? L.fwd_bytes : L.bwd_bytes;
    return L;
}

StoreTables store_tables(const pp_problem &P, const Layout &L, char *base) {
    const bool x3 = P.precision == PP_BF16X3;
    StoreTables t;
    t.xh = (const unsigned short *)(base + L.sxh);
    t.xl = x3 ? (const unsigned short *)(base + L.sxl) : nullptr;
    t.yh = (const unsigned short *)(base + L.syh);
    t.yl = x3 ? (const unsigned short *)(base + L.syl) : nullptr;
    t.ldx = store_ld(P.Mu);
    t.ldy = store_ld(P.Mp);
    return t;
}

// Work-items of one grid dimension: blocks x threads, which must stay below 2^32.
bool dim_ok(uint64_t blocks, uint64_t threads) { return blocks * threads <= 0xffffffffull; }

uint64_t cdiv(uint64_t a, uint64_t b) { return (a + b - 1) / b; }

// Every launch that any entry point may enqueue for P fits its grid (checked before any enqueue;
// the kMaxBlocks and kMaxPairs bounds keep every product here far from 64-bit overflow).
bool grids_fit(const pp_problem &P) {
    const uint64_t n = (uint64_t)P.n, MM = (uint64_t)P.Mu * (uint64_t)P.Mp;
    const FwdPlan f = fwd_plan(P);
    const BwdPlan b = bwd_plan(P);
    const bool bf = is_gen(P.precision);
    const uint64_t tiles = (uint64_t)f.tiles_u * (uint64_t)f.tiles_p;
    bool ok = dim_ok(tiles, 256) && (uint64_t)f.splits <= 0xffffffffull;
    ok = ok && dim_ok((uint64_t)reduce_scale_blocks(P.Mu, P.Mp), 256);   // split-K reduction
    ok = ok && dim_ok(cdiv(MM, 256), 256);                                 // row-form operands (FP64 / FP32)
    ok = ok && dim_ok(cdiv(n, 256), 256);                                  // final per-block sums
    if (bf) {
        ok = ok && dim_ok(cdiv((uint64_t)phase_rows(P.n), 256), 256);
        for (int axis = 0; axis < 2; ++axis) {
            const int Nb = axis == 0 ? P.Mu : P.Mp, Ka = axis == 0 ? P.Mp : P.Mu;
            const uint64_t elems = bwd_bf16_operand_elems((Nb + 255) / 256 * 256, bf16_kh(Ka));
            ok = ok && dim_ok(cdiv(elems, 256), 256);                       // tiled gradient operands
        }
        ok = ok && dim_ok(cdiv(n, 256), 512) && (uint64_t)b.tiles_nx <= 65535 && (uint64_t)b.tiles_ny <= 65535;
        if (P.basis_mode == PP_BASIS_STORE) {
            const uint64_t rows = (uint64_t)store_rows(P.n);
            const uint64_t tb = cdiv(cdiv(n, 256), 8) * 8;
            for (int M : {P.Mu, P.Mp}) {
                ok = ok && dim_ok(cdiv(rows * ((uint64_t)store_ld(M) / 32), 256), 256);   // table build
                ok = ok && dim_ok(tb * cdiv((uint64_t)M, 256), 512);                      // gradient from tables
            }
            ok = ok && dim_ok(tiles * cdiv((uint64_t)f.splits, 8) * 8, 512);               // forward from tables
        }
    } else {
        ok = ok && dim_ok(cdiv(n, (uint64_t)b.tb), 256) && (uint64_t)b.tiles_nx <= 65535 &&
             (uint64_t)b.tiles_ny <= 65535;
    }
    return ok;
}

int check_ws(const Layout &L, void *ws, size_t ws_bytes) {
    if (ws_bytes < L.total) return PP_ERR_WORKSPACE;
    if (L.total > 0 && (!ws || ((uintptr_t)ws % kAlign) != 0)) return PP_ERR_ARG;
    return PP_OK;
}

// Forward pipeline: partial contractions -> coefficients (+ energy partials) -> energy.  With
// timed = false no launch is ever bracketed by timing events.
int run_forward(const pp_problem &P, const double *x, const double *y, const double *w, const double *h,
                double *a, double *E, void *ws, hipStream_t s, bool timed = true) {
    auto T = [timed](const char *name) { return timed ? name : nullptr; };
    const FwdPlan f = fwd_plan(P);
    const Layout L = layout(P);
    char *base = (char *)ws;
    void *part = base + L.part;
    double *epart = (double *)(base + L.epart);
    hipError_t err;
    if (is_gen(P.precision)) {
        const bool x3 = P.precision == PP_BF16X3 || P.precision == PP_FP8X3;
        PhaseRec *tx = (PhaseRec *)(base + L.tx), *ty = (PhaseRec *)(base + L.ty);
        RunSeed *sx = (RunSeed *)(base + L.sdx), *sy = (RunSeed *)(base + L.sdy);
        { TimedLaunch t(T("tables"), s); err = launch_phase_tables(P.n, x, y, w, h, P.W, P.H, tx, ty, s); }
        if (err != hipSuccess) return PP_ERR_DEVICE;
        {
            TimedLaunch t(T("seeds"), s);
            err = launch_seed_table(P.n, seed_runs(P.Mu), tx, sx, s);
            if (err == hipSuccess) err = launch_seed_table(P.n, seed_runs(P.Mp), ty, sy, s);
        }
        if (err != hipSuccess) return PP_ERR_DEVICE;
        if (P.basis_mode == PP_BASIS_STORE) {
            const StoreTables st = store_tables(P, L, base);
            {
                TimedLaunch t(T("build"), s);
                err = launch_build_table(x3, P.n, P.Mu, tx, sx, (unsigned short *)st.xh, (unsigned short *)st.xl, s);
                if (err == hipSuccess)
                    err = launch_build_table(x3, P.n, P.Mp, ty, sy, (unsigned short *)st.yh, (unsigned short *)st.yl,
                                             s);
            }
            if (err != hipSuccess) return PP_ERR_DEVICE;
            { TimedLaunch t(T("fwd"), s); err = launch_fwd_bf16_st(f, x3, P.n, P.Mu, P.Mp, st, (float *)part, s); }
        } else if (is_fp8(P.precision)) {
            TimedLaunch t(T("fwd"), s);
            err = launch_fwd_fp8(f, x3, P.n, P.Mu, P.Mp, tx, ty, sx, sy, (float *)part, s);
        } else if (P.precision == PP_BF16MIX) {
            TimedLaunch t(T("fwd"), s);
            err = launch_fwd_bf16_mix(f, mix_tiles(P.Mu), mix_tiles(P.Mp), P.n, P.Mu, P.Mp, tx, ty, sx, sy,
                                      (float *)part, s);
        } else {
            TimedLaunch t(T("fwd"), s);
            err = launch_fwd_bf16(f, x3, P.n, P.Mu, P.Mp, tx, ty, sx, sy, (float *)part, s);
        }
    } else if (P.precision == PP_FP32) {
        TimedLaunch t(T("fwd"), s);
        err = launch_fwd_f32(f, P.n, P.Mu, P.Mp, P.W, P.H, x, y, w, h, (float *)part, s);
    } else {
        TimedLaunch t(T("fwd"), s);
        err = launch_fwd_f64(f, P.n, P.Mu, P.Mp, P.W, P.H, x, y, w, h, (double *)part, s);
    }
    if (err != hipSuccess) return PP_ERR_DEVICE;
    int nb = 0;
    { TimedLaunch t(T("reduce"), s); err = launch_reduce_scale(part, f.part_elem == 4, f.splits, P.Mu, P.Mp, P.W, P.H, a, epart, &nb, s); }
    if (err != hipSuccess) return PP_ERR_DEVICE;
    if (E) {
        { TimedLaunch t(T("energy"), s); err = launch_energy_final(epart, nb, E, s); }
        if (err != hipSuccess) return PP_ERR_DEVICE;
    }
    return PP_OK;
}

// Device address of `scratch` on each device, resolved once per device with that device current.
constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_addr[kMaxScratchDevices] = {};

int scratch_on_current_device(void **out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxScratchDevices) return PP_ERR_DEVICE;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_addr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return PP_ERR_DEVICE;
        g_scratch_addr[dev] = p;
    }
    *out = g_scratch_addr[dev];
    return PP_OK;
}

// FP64 / FP32 row-form contractions (FP32 operands for PP_FP32, FP64 otherwise).
hipError_t prep_rowform(const pp_problem &P, RowForm f, const double *a, void *bx, void *by, hipStream_t s) {
    TimedLaunch t("prep", s);
    if (P.precision == PP_FP32)
        return launch_prep_rowform_f32(f, a, P.Mu, P.Mp, P.W, P.H, (float *)bx, (float *)by, s);
    return launch_prep_rowform_f64(f, a, P.Mu, P.Mp, P.W, P.H, (double *)bx, (double *)by, s);
}

hipError_t rowform(const pp_problem &P, RowForm f, const BwdPlan &b, const BwdAxis &ax, hipStream_t s) {
    return P.precision == PP_FP32 ? launch_rowform_f32(f, b, P.n, ax, s) : launch_rowform_f64(f, b, P.n, ax, s);
}

}  // namespace
}  // namespace pp

using namespace pp;

extern "C" {

int pp_workspace_size(const pp_problem *P, size_t *bytes) {
    const int st = validate_problem(P);
    if (st != PP_OK) return st;
    if (!bytes) return PP_ERR_ARG;
    *bytes = layout(*P).total;
    return PP_OK;
}

int pp_coeffs(const pp_problem *P, const double *x, const double *y, const double *w, const double *h, double *a,
              void *ws, size_t ws_bytes, void *stream) {
    int st = validate_problem(P);
    if (st != PP_OK) return st;
    if ((st = validate_blocks(P, x, y, w, h)) != PP_OK) return st;
    if (!a || !aligned8(a)) return PP_ERR_ARG;
    const Layout L = layout(*P);
    if ((st = check_ws(L, ws, ws_bytes)) != PP_OK) return st;
    return run_forward(*P, x, y, w, h, a, nullptr, ws, (hipStream_t)stream);
}

int pp_energy(const pp_problem *P, const double *x, const double *y, const double *w, const double *h, double *E,
              double *a, void *ws, size_t ws_bytes, void *stream) {
    int st = validate_problem(P);
    if (st != PP_OK) return st;
    if ((st = validate_blocks(P, x, y, w, h)) != PP_OK) return st;
    if (!E || !aligned8(E) || (a && !aligned8(a))) return PP_ERR_ARG;
    const Layout L = layout(*P);
    if ((st = check_ws(L, ws, ws_bytes)) != PP_OK) return st;
    return run_forward(*P, x, y, w, h, a, E, ws, (hipStream_t)stream);
}

int pp_energy_static(const pp_problem *P, const double *x, const double *y, const double *w, const double *h,
                     double *E, double *a, void *stream) {
    int st = validate_problem(P);
    if (st != PP_OK) return st;
    if (P->basis_mode != PP_BASIS_RECOMPUTE) return PP_ERR_UNSUPPORTED;
    if ((st = validate_blocks(P, x, y, w, h)) != PP_OK) return st;
    if (!E || !aligned8(E) || (a && !aligned8(a))) return PP_ERR_ARG;
    const Layout L = layout(*P);
    if (L.total > (size_t)PP_STATIC_SCRATCH_BYTES) return PP_ERR_SCRATCH;
    void *ws = nullptr;
    if ((st = scratch_on_current_device(&ws)) != PP_OK) return st;
    // Every byte of the workspace that the forward reads is written earlier in the same call (phase
    // records with their zero padding, every split's partial tile, every energy partial), so what an
    // earlier call left in the shared array needs no clearing.  No launch of this call is timed.
    return run_forward(*P, x, y, w, h, a, E, ws, (hipStream_t)stream, false);
}

int pp_field(const pp_problem *P, const double *x, const double *y, const double *w, const double *h,
             const double *a, const double *dE, double *gx, double *gy, void *ws, size_t ws_bytes, void *stream) {
    int st = validate_problem(P);
    if (st != PP_OK) return st;
    if ((st = validate_blocks(P, x, y, w, h)) != PP_OK) return st;
    if (!a || !aligned8(a) || (dE && !aligned8(dE))) return PP_ERR_ARG;
    if (P->n > 0 && (!gx || !gy || !aligned8(gx) || !aligned8(gy))) return PP_ERR_ARG;
    const Layout L = layout(*P);
    if ((st = check_ws(L, ws, ws_bytes)) != PP_OK) return st;
    if (P->n == 0) return PP_OK;
    hipStream_t s = (hipStream_t)stream;
    const BwdPlan b = bwd_plan(*P);
    char *base = (char *)ws;
    double *gpx = (double *)(base + L.gpx), *gpy = (double *)(base + L.gpy);
    if (is_fp8(P->precision)) {
        const bool x3 = P->precision == PP_FP8X3;
        PhaseRec *tx = (PhaseRec *)(base + L.tx), *ty = (PhaseRec *)(base + L.ty);
        unsigned char *bxt = (unsigned char *)(base + L.bx), *byt = (unsigned char *)(base + L.by);
        float *b0x = (float *)(base + L.b0x), *b0y = (float *)(base + L.b0y);
        const int khx = bf16_kh(P->Mp), khy = bf16_kh(P->Mu);
        { TimedLaunch t("tables", s); if (launch_phase_tables(P->n, x, y, w, h, P->W, P->H, tx, ty, s) != hipSuccess) return PP_ERR_DEVICE; }
        {
            TimedLaunch t("prep", s);
            if (launch_prep_bwd_fp8(ROW_FIELD, a, P->Mu, P->Mp, P->W, P->H, 0, b.tiles_nx * 256, khx, bxt, b0x, s) !=
                hipSuccess)
                return PP_ERR_DEVICE;
            if (launch_prep_bwd_fp8(ROW_FIELD, a, P->Mu, P->Mp, P->W, P->H, 1, b.tiles_ny * 256, khy, byt, b0y, s) !=
                hipSuccess)
                return PP_ERR_DEVICE;
        }
        // gx: K = p (basis of y), epilogue over u (x);  gy: K = u (basis of x), epilogue over p (y).
        const BwdAxisFp8 axx{ty, tx, P->Mp, P->Mu, khx, bxt, b0x, gpx, nullptr, 0.0f};
        const BwdAxisFp8 axy{tx, ty, P->Mu, P->Mp, khy, byt, b0y, gpy, nullptr, 0.0f};
        { TimedLaunch t("bwd", s); if (launch_bwd_fp8(ROW_FIELD, x3, P->n, axx, s) != hipSuccess) return PP_ERR_DEVICE; }
        { TimedLaunch t("bwd", s); if (launch_bwd_fp8(ROW_FIELD, x3, P->n, axy, s) != hipSuccess) return PP_ERR_DEVICE; }
        { TimedLaunch t("final", s); if (launch_bwd_final(gpx, b.tiles_nx, gpy, b.tiles_ny, P->n, dE, gx, gy, s) != hipSuccess) return PP_ERR_DEVICE; }
        return PP_OK;
    }
    if (is_bf16(P->precision)) {
        const bool x3 = P->precision == PP_BF16X3;
        PhaseRec *tx = (PhaseRec *)(base + L.tx), *ty = (PhaseRec *)(base + L.ty);
        unsigned short *bxt = (unsigned short *)(base + L.bx), *byt = (unsigned short *)(base + L.by);
        const int khx = bf16_kh(P->Mp), khy = bf16_kh(P->Mu);
        { TimedLaunch t("tables", s); if (launch_phase_tables(P->n, x, y, w, h, P->W, P->H, tx, ty, s) != hipSuccess) return PP_ERR_DEVICE; }
        {
            TimedLaunch t("prep", s);
            if (launch_prep_bwd_bf16(ROW_FIELD, a, P->Mu, P->Mp, P->W, P->H, 0, b.tiles_nx * 256, khx, bxt, s) !=
                hipSuccess)
                return PP_ERR_DEVICE;
            if (launch_prep_bwd_bf16(ROW_FIELD, a, P->Mu, P->Mp, P->W, P->H, 1, b.tiles_ny * 256, khy, byt, s) !=
                hipSuccess)
                return PP_ERR_DEVICE;
        }
        // gx: K = p (basis of y), epilogue over u (x);  gy: K = u (basis of x), epilogue over p (y).
        BwdAxisBf16 axx{ty, tx, P->Mp, P->Mu, khx, bxt, gpx, nullptr, nullptr, 0, 0, 0, nullptr, 0.0f};
        BwdAxisBf16 axy{tx, ty, P->Mu, P->Mp, khy, byt, gpy, nullptr, nullptr, 0, 0, 0, nullptr, 0.0f};
        if (P->basis_mode == PP_BASIS_STORE) {
            // the tables that pp_coeffs / pp_energy left in the workspace
            const StoreTables st = store_tables(*P, L, base);
            const int tb = (int)((P->n + 255) / 256);
            axx.tab_h = st.yh; axx.tab_l = st.yl; axx.tab_ld = st.ldy;
            axx.tiles_b = tb; axx.tiles_n = (P->Mu + 255) / 256;
            axy.tab_h = st.xh; axy.tab_l = st.xl; axy.tab_ld = st.ldx;
            axy.tiles_b = tb; axy.tiles_n = (P->Mp + 255) / 256;
        }
        if (P->precision == PP_BF16MIX) {
            // the low-frequency N tiles with three products, the others with one (the K axis whole in
            // both); each launch writes the partial row sums of its own N tiles
            const int rx = mix_tiles(P->Mu), ry = mix_tiles(P->Mp);
            for (int axis = 0; axis < 2; ++axis) {
                TimedLaunch t("bwd", s);
                BwdAxisBf16 lo = axis == 0 ? axx : axy, hi = lo;
                const int r = axis == 0 ? rx : ry, tn = axis == 0 ? b.tiles_nx : b.tiles_ny;
                lo.nt0 = 0; lo.nt_end = r;
                if (launch_bwd_bf16(ROW_FIELD, true, P->n, lo, s) != hipSuccess) return PP_ERR_DEVICE;
                if (r < tn) {
                    hi.nt0 = r; hi.nt_end = tn;
                    if (launch_bwd_bf16(ROW_FIELD, false, P->n, hi, s) != hipSuccess) return PP_ERR_DEVICE;
                }
            }
        } else {
            { TimedLaunch t("bwd", s); if (launch_bwd_bf16(ROW_FIELD, x3, P->n, axx, s) != hipSuccess) return PP_ERR_DEVICE; }
            { TimedLaunch t("bwd", s); if (launch_bwd_bf16(ROW_FIELD, x3, P->n, axy, s) != hipSuccess) return PP_ERR_DEVICE; }
        }
        { TimedLaunch t("final", s); if (launch_bwd_final(gpx, b.tiles_nx, gpy, b.tiles_ny, P->n, dE, gx, gy, s) != hipSuccess) return PP_ERR_DEVICE; }
        return PP_OK;
    }
    void *bx = base + L.bx, *by = base + L.by;
    if (prep_rowform(*P, ROW_FIELD, a, bx, by, s) != hipSuccess) return PP_ERR_DEVICE;
    // gx: K = p (basis of y), epilogue over u (cosine differences of x), operand BxT[p][u].
    BwdAxis axx{y, h, P->H, P->Mp, x, w, P->W, P->Mu, bx, gpx, nullptr};
    // gy: K = u (basis of x), epilogue over p (cosine differences of y), operand By[u][p].
    BwdAxis axy{x, w, P->W, P->Mu, y, h, P->H, P->Mp, by, gpy, nullptr};
    { TimedLaunch t("bwd", s); if (rowform(*P, ROW_FIELD, b, axx, s) != hipSuccess) return PP_ERR_DEVICE; }
    { TimedLaunch t("bwd", s); if (rowform(*P, ROW_FIELD, b, axy, s) != hipSuccess) return PP_ERR_DEVICE; }
    { TimedLaunch t("final", s); if (launch_bwd_final(gpx, b.tiles_nx, gpy, b.tiles_ny, P->n, dE, gx, gy, s) != hipSuccess) return PP_ERR_DEVICE; }
    return PP_OK;
}

int pp_point_field(const pp_problem *P, const double *px, const double *py, const double *a, double *psi,
                   double *xix, double *xiy, void *ws, size_t ws_bytes, void *stream) {
    int st = validate_problem(P);
    if (st != PP_OK) return st;
    if (P->basis_mode != PP_BASIS_RECOMPUTE || is_fp8(P->precision) || P->precision == PP_BF16MIX)
        return PP_ERR_UNSUPPORTED;
    if (P->n > 0 && (!px || !py || !aligned8(px) || !aligned8(py))) return PP_ERR_ARG;
    if (!a || !aligned8(a)) return PP_ERR_ARG;
    if ((psi && !aligned8(psi)) || (xix && !aligned8(xix)) || (xiy && !aligned8(xiy))) return PP_ERR_ARG;
    const Layout L = layout(*P);
    if ((st = check_ws(L, ws, ws_bytes)) != PP_OK) return st;
    if (P->n == 0 || (!psi && !xix && !xiy)) return PP_OK;
    hipStream_t s = (hipStream_t)stream;
    const BwdPlan b = bwd_plan(*P);
    char *base = (char *)ws;
    double *gp1 = (double *)(base + L.gpx), *gp2 = (double *)(base + L.gpz), *gpy = (double *)(base + L.gpy);
    void *bx = base + L.bx, *by = base + L.by;
    if (is_bf16(P->precision)) {
        // bf16 operands: point phase records (size 0), hi/lo tiled a, the bf16 row-form kernels.
        const bool x3 = P->precision == PP_BF16X3;
        PhaseRec *tx = (PhaseRec *)(base + L.tx), *ty = (PhaseRec *)(base + L.ty);
        unsigned short *bxt = (unsigned short *)bx, *byt = (unsigned short *)by;
        const int khx = bf16_kh(P->Mp), khy = bf16_kh(P->Mu);
        { TimedLaunch t("tables", s); if (launch_phase_tables(P->n, px, py, nullptr, nullptr, P->W, P->H, tx, ty, s) != hipSuccess) return PP_ERR_DEVICE; }
        {
            TimedLaunch t("prep", s);
            if ((psi || xix) &&
                launch_prep_bwd_bf16(ROW_POINT_DUAL, a, P->Mu, P->Mp, P->W, P->H, 0, b.tiles_nx * 256, khx, bxt, s) !=
                    hipSuccess)
                return PP_ERR_DEVICE;
            if (xiy &&
                launch_prep_bwd_bf16(ROW_POINT_DUAL, a, P->Mu, P->Mp, P->W, P->H, 1, b.tiles_ny * 256, khy, byt, s) !=
                    hipSuccess)
                return PP_ERR_DEVICE;
        }
        if (psi || xix) {
            TimedLaunch t("point", s);
            const RowForm f = psi ? ROW_POINT_DUAL : ROW_POINT_WSIN;
            BwdAxisBf16 ax{ty, tx, P->Mp, P->Mu, khx, bxt, psi ? gp1 : gp2, nullptr, nullptr, 0, 0, 0,
                           psi ? gp2 : nullptr, (float)(kPi / P->W)};
            if (launch_bwd_bf16(f, x3, P->n, ax, s) != hipSuccess) return PP_ERR_DEVICE;
        }
        if (xiy) {
            TimedLaunch t("point", s);
            BwdAxisBf16 ax{tx, ty, P->Mu, P->Mp, khy, byt, gpy, nullptr, nullptr, 0, 0, 0, nullptr, (float)(kPi / P->H)};
            if (launch_bwd_bf16(ROW_POINT_WSIN, x3, P->n, ax, s) != hipSuccess) return PP_ERR_DEVICE;
        }
        TimedLaunch t("final", s);
        if (launch_bwd_final(gp1, b.tiles_nx, gpy, b.tiles_ny, P->n, nullptr, psi, xiy, s) != hipSuccess)
            return PP_ERR_DEVICE;
        if (xix && launch_bwd_final(gp2, b.tiles_nx, gp2, 0, P->n, nullptr, xix, nullptr, s) != hipSuccess)
            return PP_ERR_DEVICE;
        return PP_OK;
    }
    if (prep_rowform(*P, ROW_POINT_DUAL, a, bx, xiy ? by : nullptr, s) != hipSuccess) return PP_ERR_DEVICE;
    // psi and xi_x share Z_iu = sum_p a_up cos(v_p y_i) (K = p, operand a^T); epilogues over u with
    // cos(w_u x_i) and w_u sin(w_u x_i).
    if (psi || xix) {
        TimedLaunch t("point", s);
        const RowForm f = psi ? ROW_POINT_DUAL : ROW_POINT_WSIN;
        BwdAxis ax{py, nullptr, P->H, P->Mp, px, nullptr, P->W, P->Mu, bx, psi ? gp1 : gp2, psi ? gp2 : nullptr};
        if (rowform(*P, f, b, ax, s) != hipSuccess) return PP_ERR_DEVICE;
    }
    // xi_y: K = u with cos(w_u x_i), operand a[u][p], epilogue over p with v_p sin(v_p y_i).
    if (xiy) {
        TimedLaunch t("point", s);
        BwdAxis ax{px, nullptr, P->W, P->Mu, py, nullptr, P->H, P->Mp, by, gpy, nullptr};
        if (rowform(*P, ROW_POINT_WSIN, b, ax, s) != hipSuccess) return PP_ERR_DEVICE;
    }
    TimedLaunch t("final", s);
    if (launch_bwd_final(gp1, b.tiles_nx, gpy, b.tiles_ny, P->n, nullptr, psi, xiy, s) != hipSuccess)
        return PP_ERR_DEVICE;
    if (xix && launch_bwd_final(gp2, b.tiles_nx, gp2, 0, P->n, nullptr, xix, nullptr, s) != hipSuccess)
        return PP_ERR_DEVICE;
    return PP_OK;
}

int pp_block_potential(const pp_problem *P, const double *x, const double *y, const double *w, const double *h,
                       const double *a, double *N, void *ws, size_t ws_bytes, void *stream) {
    int st = validate_problem(P);
    if (st != PP_OK) return st;
    if (P->basis_mode != PP_BASIS_RECOMPUTE || is_fp8(P->precision) || P->precision == PP_BF16MIX)
        return PP_ERR_UNSUPPORTED;
    if ((st = validate_blocks(P, x, y, w, h)) != PP_OK) return st;
    if (!a || !aligned8(a)) return PP_ERR_ARG;
    if (P->n > 0 && (!N || !aligned8(N))) return PP_ERR_ARG;
    const Layout L = layout(*P);
    if ((st = check_ws(L, ws, ws_bytes)) != PP_OK) return st;
    if (P->n == 0) return PP_OK;
    hipStream_t s = (hipStream_t)stream;
    const BwdPlan b = bwd_plan(*P);
    char *base = (char *)ws;
    double *gp = (double *)(base + L.gpx);
    void *bx = base + L.bx;
    if (is_bf16(P->precision)) {
        const bool x3 = P->precision == PP_BF16X3;
        PhaseRec *tx = (PhaseRec *)(base + L.tx), *ty = (PhaseRec *)(base + L.ty);
        unsigned short *bxt = (unsigned short *)bx;
        const int khx = bf16_kh(P->Mp);
        { TimedLaunch t("tables", s); if (launch_phase_tables(P->n, x, y, w, h, P->W, P->H, tx, ty, s) != hipSuccess) return PP_ERR_DEVICE; }
        {
            TimedLaunch t("prep", s);
            if (launch_prep_bwd_bf16(ROW_POTENTIAL, a, P->Mu, P->Mp, P->W, P->H, 0, b.tiles_nx * 256, khx, bxt, s) !=
                hipSuccess)
                return PP_ERR_DEVICE;
        }
        {
            TimedLaunch t("potential", s);
            BwdAxisBf16 ax{ty, tx, P->Mp, P->Mu, khx, bxt, gp, nullptr, nullptr, 0, 0, 0, nullptr, 0.0f};
            if (launch_bwd_bf16(ROW_POTENTIAL, x3, P->n, ax, s) != hipSuccess) return PP_ERR_DEVICE;
        }
        TimedLaunch t("final", s);
        if (launch_bwd_final(gp, b.tiles_nx, gp, 0, P->n, nullptr, N, nullptr, s) != hipSuccess) return PP_ERR_DEVICE;
        return PP_OK;
    }
    if (prep_rowform(*P, ROW_POTENTIAL, a, bx, nullptr, s) != hipSuccess) return PP_ERR_DEVICE;
    // N_i = sum_u S_iu sum_p T_ip a_up / (vt_p wt_u): K = p, epilogue over u, both sine differences.
    {
        TimedLaunch t("potential", s);
        BwdAxis ax{y, h, P->H, P->Mp, x, w, P->W, P->Mu, bx, gp, nullptr};
        if (rowform(*P, ROW_POTENTIAL, b, ax, s) != hipSuccess) return PP_ERR_DEVICE;
    }
    TimedLaunch t("final", s);
    if (launch_bwd_final(gp, b.tiles_nx, gp, 0, P->n, nullptr, N, nullptr, s) != hipSuccess) return PP_ERR_DEVICE;
    return PP_OK;
}

const char *pp_strerror(int status) {
    switch (status) {
        case PP_OK: return "success";
        case PP_ERR_ARG: return "invalid argument (NULL or misaligned pointer, bad size, non-finite or non-positive region)";
        case PP_ERR_WORKSPACE: return "workspace smaller than pp_workspace_size()";
        case PP_ERR_UNSUPPORTED: return "precision or basis mode not implemented by the library";
        case PP_ERR_DEVICE: return "HIP launch or runtime error";
        case PP_ERR_SCRATCH: return "problem needs more workspace than the static scratch (PP_STATIC_SCRATCH_BYTES)";
        default: return "unknown status";
    }
}

}  // extern "C"
