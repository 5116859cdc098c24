/*
 * pp_oracle.c -- FP64 oracle for the truncated analytical cosine-series solution of
 * Poisson's equation with Neumann boundary conditions, driven by the exact rectangle
 * block density (arXiv 2307.12041, Sec. III-A).
 *
 * TEST INFRASTRUCTURE ONLY.  This code is the independent checker of the GPU library.
 * Only the tests, the smoke check and the CPU-baseline leg of the benchmark load it.
 * The GPU library never calls it, and it shares no code, header, table or constant
 * with the GPU path.
 *
 * What it computes, by plain direct summation in double precision (sums over blocks
 * accumulated in long double, in block order, so the result does not depend on the
 * thread count):
 *
 *  1. Sine and cosine differences of the block edges.  For block i with centre x_i and
 *     width w_i, and frequency index u >= 1,
 *         S_iu = sin(u pi (x_i + w_i/2) / W) - sin(u pi (x_i - w_i/2) / W),
 *         K_iu = cos(u pi (x_i + w_i/2) / W) - cos(u pi (x_i - w_i/2) / W),
 *     and T_ip, L_ip the same in y with h_i, H (the bracketed factors of the closed-form
 *     coefficients, Sec. III-A, eqs. for a_{mu,eta}, a_{mu,0}, a_{0,eta}).  Arguments
 *     are reduced exactly: u*t = P + e by an FMA two-product, P reduced modulo 2W by
 *     fmod (exact), phase = pi*(P mod 2W + e)/W, then libm sin/cos.
 *
 *  2. The coefficients, case by case (Sec. III-A, coefficient summary and the three
 *     closed forms derived from the mean-subtracted exact density):
 *         a_00 = 0,
 *         a_u0 = 2 W^2 / (u^3 pi^3 H) * sum_i h_i S_iu,
 *         a_0p = 2 H^2 / (p^3 pi^3 W) * sum_i w_i T_ip,
 *         a_up = 4 W^2 H^2 / ((u^2 H^2 + p^2 W^2) u p pi^4) * sum_i S_iu T_ip.
 *     The cosine moments of the density, I_up = iint_R rho cos(u pi x/W) cos(p pi y/H),
 *     follow from the same sums: I_u0 = W/(u pi) sum h S, I_0p = H/(p pi) sum w T,
 *     I_up = W H/(u p pi^2) sum S T, and I_00 = 0 after the mean subtraction.
 *
 *  3. The energy E = 1/2 iint_R rho psi = 1/2 sum_up a_up I_up (the electrostatic
 *     energy of Sec. II-B, N = 1/2 sum_i q_i psi_i, read with the exact block density:
 *     every block contributes its charge density times the potential over its area).
 *
 *  4. The gradient of E with respect to block centres:
 *         dE/dx_i = sum_{u>=1} sum_p a_up K_iu Ybar_ip,  dE/dy_i = sum_u sum_{p>=1} a_up Xbar_iu L_ip,
 *     with Xbar_iu = W/(u pi) S_iu (u >= 1), Xbar_i0 = w_i, and Ybar likewise.  It equals
 *     minus the field of eq. (ksi) integrated over block i.
 *
 *  5. Point values of the potential psi (eq. psi) and field xi (eq. ksi), and the block
 *     potentials N_i = iint_{block i} psi = sum_up a_up Xbar_iu Ybar_ip.
 *
 *  6. The bin scheme of Sec. III-D (a comparison path): an m x m grid of bins of size
 *     wb = W/m, hb = H/m with centres x_l = (l + 1/2) wb, y_j = (j + 1/2) hb;
 *       - bin densities P_lj = (area of the blocks inside bin lj) / (wb hb), read as the exact
 *         overlap areas (the paper's "local smoothness" is not specified and is not applied);
 *       - the binned coefficients of eqs. disa-a..d, i.e. the coefficients of the density
 *         sum_lj P_lj [bin lj] minus its mean (eq. rho-dis), as plain double sums over the bins:
 *           a_00 = 0,
 *           a_0p = 4 H^2 / (p^3 pi^3 m) sin(p pi/(2m)) sum_lj P_lj cos(p (j+1/2) pi/m),
 *           a_u0 = 4 W^2 / (u^3 pi^3 m) sin(u pi/(2m)) sum_lj P_lj cos(u (l+1/2) pi/m),
 *           a_up = 16 W^2 H^2 / (u p (u^2 H^2 + p^2 W^2) pi^4) sin(u pi/(2m)) sin(p pi/(2m))
 *                  * sum_lj P_lj cos(u (l+1/2) pi/m) cos(p (j+1/2) pi/m)
 *         (the cosine argument of eq. disa-c, garbled in the text, is read as u (l + 1/2) pi/m);
 *       - the potential and field at the bin centres truncated at the coefficient array
 *         (eqs. dis-psi1 and dis-ksi):
 *           psi(l,j) = sum_up a_up cos(u (l+1/2) pi/m) cos(p (j+1/2) pi/m),
 *           xi_x(l,j) = sum_up (u pi/W) a_up sin(u (l+1/2) pi/m) cos(p (j+1/2) pi/m),
 *           xi_y(l,j) = sum_up (p pi/H) a_up cos(u (l+1/2) pi/m) sin(p (j+1/2) pi/m).
 *     Cosines and sines of k (2l+1) pi/(2m) take the integer k (2l+1) modulo 4m first;
 *       - the values of each block from those of the bins around it (the last step of the
 *         scheme, whose weights the paper leaves open), read as the integral over the block of
 *         the bin values held constant on each bin, in the conventions of item 5 and of item 4:
 *           N_i  = sum_lj |block i cap bin lj| psi(l,j),
 *           gx_i = - sum_lj |block i cap bin lj| xi_x(l,j),  gy_i = - sum_lj ... xi_y(l,j),
 *         the counterparts of the block potentials and of the gradient of the direct path.
 *
 * Truncation: u in [0, Mu), p in [0, Mp).  Coefficient arrays are row-major, a[u*Mp + p].
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_PI 3.14159265358979323846264338327950288

/* sin and cos of pi*k*t/L, with k*t reduced modulo 2L exactly. */
static void sincos_kpi(long k, double t, double L, double *s, double *c)
{
    double kd = (double)k;
    double P = kd * t;
    double e = fma(kd, t, -P);          /* k*t = P + e exactly */
    double r = fmod(P, 2.0 * L);        /* exact */
    double phi = ORACLE_PI * ((r + e) / L);
    *s = sin(phi);
    *c = cos(phi);
}

/* S (sine difference) and K (cosine difference) of one block edge pair at frequency k. */
static void edge_diffs(long k, double centre, double size, double L, double *S, double *K)
{
    double sp, cp, sm, cm;
    sincos_kpi(k, centre + size / 2.0, L, &sp, &cp);
    sincos_kpi(k, centre - size / 2.0, L, &sm, &cm);
    *S = sp - sm;
    *K = cp - cm;
}

/* Integral of cos(k pi t / L) over the block extent: L/(k pi) * S for k >= 1, size for k = 0. */
static double edge_integral(long k, double centre, double size, double L)
{
    if (k == 0) return size;
    double S, K;
    edge_diffs(k, centre, size, L, &S, &K);
    return L / ((double)k * ORACLE_PI) * S;
}

void oracle_set_num_threads(int k)
{
#ifdef _OPENMP
    if (k > 0) omp_set_num_threads(k);
#else
    (void)k;
#endif
}

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Coefficient prefactor of the three closed forms, and the moment prefactor. */
static double coef_factor(long u, long p, double W, double H)
{
    const double pi = ORACLE_PI;
    if (u == 0 && p == 0) return 0.0;
    if (p == 0) return 2.0 * W * W / ((double)u * u * u * pi * pi * pi * H);
    if (u == 0) return 2.0 * H * H / ((double)p * p * p * pi * pi * pi * W);
    return 4.0 * W * W * H * H /
           (((double)u * u * H * H + (double)p * p * W * W) * (double)u * (double)p * pi * pi * pi * pi);
}

static double moment_factor(long u, long p, double W, double H)
{
    const double pi = ORACLE_PI;
    if (u == 0 && p == 0) return 0.0;
    if (p == 0) return W / ((double)u * pi);
    if (u == 0) return H / ((double)p * pi);
    return W * H / ((double)u * (double)p * pi * pi);
}

/*
 * Raw sums R_up = sum_i S'_iu T'_ip with S'_iu = S_iu (u >= 1), S'_i0 = w_i, and T' the same
 * in y (so R_u0 = sum h S, R_0p = sum w T, R_up = sum S T).  Blocks are processed in chunks
 * to bound memory; within each (u,p) the sum runs over i in increasing order.
 */
static int raw_sums(double W, double H, int64_t n, const double *x, const double *y,
                    const double *w, const double *h, int Mu, int Mp, long double *R)
{
    const int64_t CH = 2048;
    double *Sc = (double *)malloc(sizeof(double) * (size_t)CH * (size_t)Mu);
    double *Tc = (double *)malloc(sizeof(double) * (size_t)CH * (size_t)Mp);
    if (!Sc || !Tc) { free(Sc); free(Tc); return -1; }
    memset(R, 0, sizeof(long double) * (size_t)Mu * (size_t)Mp);
    for (int64_t i0 = 0; i0 < n; i0 += CH) {
        int64_t m = (n - i0 < CH) ? (n - i0) : CH;
#pragma omp parallel for schedule(static)
        for (int64_t j = 0; j < m; ++j) {
            int64_t i = i0 + j;
            double S, K;
            Sc[j * Mu + 0] = w[i];
            for (int u = 1; u < Mu; ++u) { edge_diffs(u, x[i], w[i], W, &S, &K); Sc[j * Mu + u] = S; }
            Tc[j * Mp + 0] = h[i];
            for (int p = 1; p < Mp; ++p) { edge_diffs(p, y[i], h[i], H, &S, &K); Tc[j * Mp + p] = S; }
        }
#pragma omp parallel for schedule(dynamic, 1)
        for (int u = 0; u < Mu; ++u) {
            long double *Ru = R + (size_t)u * Mp;
            for (int64_t j = 0; j < m; ++j) {
                long double s = Sc[j * Mu + u];
                if (s == 0.0L) continue;
                const double *Tj = Tc + j * Mp;
                for (int p = 0; p < Mp; ++p) Ru[p] += s * (long double)Tj[p];
            }
        }
    }
    free(Sc);
    free(Tc);
    return 0;
}

/*
 * Coefficients a[u*Mp+p] (three cases) and, if I != NULL, the density moments I[u*Mp+p].
 * Returns 0 on success, -1 on allocation failure, -2 on bad arguments.
 */
int oracle_coeffs(double W, double H, int64_t n, const double *x, const double *y,
                  const double *w, const double *h, int Mu, int Mp, double *a, double *I)
{
    if (!(W > 0) || !(H > 0) || Mu < 1 || Mp < 1 || n < 0 || !a) return -2;
    long double *R = (long double *)malloc(sizeof(long double) * (size_t)Mu * (size_t)Mp);
    if (!R) return -1;
    if (raw_sums(W, H, n, x, y, w, h, Mu, Mp, R)) { free(R); return -1; }
    for (int u = 0; u < Mu; ++u)
        for (int p = 0; p < Mp; ++p) {
            long double r = R[(size_t)u * Mp + p];
            a[(size_t)u * Mp + p] = (double)(coef_factor(u, p, W, H) * r);
            if (I) I[(size_t)u * Mp + p] = (double)(moment_factor(u, p, W, H) * r);
        }
    free(R);
    return 0;
}

/*
 * The raw block sums R[u*Mp+p] = sum_i S'_iu T'_ip themselves (S'_i0 = w_i, T'_i0 = h_i).  They are
 * the cosine moments with the frequency factors taken out (R_up = I_up u p pi^2 / (W H) for
 * u, p >= 1, and likewise for the axis rows), so their magnitude does not fall with (u, p): every
 * part of the (u, p) plane weighs alike in a comparison.  R_00 = sum w h (no mean subtraction here).
 */
int oracle_raw_moments(double W, double H, int64_t n, const double *x, const double *y,
                       const double *w, const double *h, int Mu, int Mp, double *Rout)
{
    if (!(W > 0) || !(H > 0) || Mu < 1 || Mp < 1 || n < 0 || !Rout) return -2;
    long double *R = (long double *)malloc(sizeof(long double) * (size_t)Mu * (size_t)Mp);
    if (!R) return -1;
    if (raw_sums(W, H, n, x, y, w, h, Mu, Mp, R)) { free(R); return -1; }
    for (size_t k = 0; k < (size_t)Mu * (size_t)Mp; ++k) Rout[k] = (double)R[k];
    free(R);
    return 0;
}

/* The prefactors f[u*Mp+p] of the three closed forms, a_up = f_up R_up (f_00 = 0). */
int oracle_coef_factors(double W, double H, int Mu, int Mp, double *f)
{
    if (!(W > 0) || !(H > 0) || Mu < 1 || Mp < 1 || !f) return -2;
    for (int u = 0; u < Mu; ++u)
        for (int p = 0; p < Mp; ++p) f[(size_t)u * Mp + p] = coef_factor(u, p, W, H);
    return 0;
}

/* E = 1/2 sum_up a_up I_up. */
double oracle_energy_from(const double *a, const double *I, int Mu, int Mp)
{
    long double e = 0.0L;
    for (size_t k = 0; k < (size_t)Mu * (size_t)Mp; ++k) e += (long double)a[k] * (long double)I[k];
    return (double)(0.5L * e);
}

/* Coefficients, moments (optional) and energy in one call. */
int oracle_energy(double W, double H, int64_t n, const double *x, const double *y,
                  const double *w, const double *h, int Mu, int Mp, double *E, double *a, double *I)
{
    size_t MM = (size_t)Mu * (size_t)Mp;
    double *aa = a ? a : (double *)malloc(sizeof(double) * MM);
    double *II = I ? I : (double *)malloc(sizeof(double) * MM);
    int st = (aa && II) ? oracle_coeffs(W, H, n, x, y, w, h, Mu, Mp, aa, II) : -1;
    if (st == 0 && E) *E = oracle_energy_from(aa, II, Mu, Mp);
    if (!a) free(aa);
    if (!I) free(II);
    return st;
}

/* Gradient of one block, given the coefficients a.  Work arrays: Mu + Mp doubles each for
 * the integrals and the cosine differences. */
static void grad_one(double W, double H, double xi, double yi, double wi, double hi,
                     int Mu, int Mp, const double *a, double *Xb, double *Kx, double *Yb, double *Ly,
                     double *gx, double *gy)
{
    for (int u = 0; u < Mu; ++u) {
        if (u == 0) { Xb[0] = wi; Kx[0] = 0.0; continue; }
        double S, K;
        edge_diffs(u, xi, wi, W, &S, &K);
        Xb[u] = W / ((double)u * ORACLE_PI) * S;
        Kx[u] = K;
    }
    for (int p = 0; p < Mp; ++p) {
        if (p == 0) { Yb[0] = hi; Ly[0] = 0.0; continue; }
        double S, K;
        edge_diffs(p, yi, hi, H, &S, &K);
        Yb[p] = H / ((double)p * ORACLE_PI) * S;
        Ly[p] = K;
    }
    long double sx = 0.0L, sy = 0.0L;
    for (int u = 0; u < Mu; ++u) {
        const double *au = a + (size_t)u * Mp;
        long double zy = 0.0L, zl = 0.0L;
        for (int p = 0; p < Mp; ++p) {
            zy += (long double)au[p] * Yb[p];   /* sum_p a_up Ybar_ip */
            zl += (long double)au[p] * Ly[p];   /* sum_p a_up L_ip */
        }
        sx += Kx[u] * zy;
        sy += Xb[u] * zl;
    }
    *gx = (double)sx;
    *gy = (double)sy;
}

static int grad_list(double W, double H, const double *x, const double *y, const double *w,
                     const double *h, int Mu, int Mp, const double *a, int64_t nb, const int64_t *idx,
                     double *gx, double *gy)
{
    int fail = 0;
#pragma omp parallel
    {
        double *buf = (double *)malloc(sizeof(double) * (size_t)(2 * Mu + 2 * Mp));
        if (!buf) {
#pragma omp atomic write
            fail = 1;
        }
#pragma omp for schedule(dynamic, 16)
        for (int64_t j = 0; j < nb; ++j) {
            if (!buf) continue;
            int64_t i = idx ? idx[j] : j;
            grad_one(W, H, x[i], y[i], w[i], h[i], Mu, Mp, a, buf, buf + Mu, buf + 2 * Mu,
                     buf + 2 * Mu + Mp, &gx[j], &gy[j]);
        }
        free(buf);
    }
    return fail ? -1 : 0;
}

/* dE/dx_i, dE/dy_i for all n blocks, given a = oracle coefficients of the same blocks. */
int oracle_grad(double W, double H, int64_t n, const double *x, const double *y, const double *w,
                const double *h, int Mu, int Mp, const double *a, double *gx, double *gy)
{
    if (!(W > 0) || !(H > 0) || Mu < 1 || Mp < 1 || n < 0) return -2;
    return grad_list(W, H, x, y, w, h, Mu, Mp, a, n, NULL, gx, gy);
}

/* The same for the listed blocks only (gx[j], gy[j] belong to block idx[j]). */
int oracle_grad_sampled(double W, double H, const double *x, const double *y, const double *w,
                        const double *h, int Mu, int Mp, const double *a, int64_t nb,
                        const int64_t *idx, double *gx, double *gy)
{
    if (!(W > 0) || !(H > 0) || Mu < 1 || Mp < 1 || nb < 0) return -2;
    return grad_list(W, H, x, y, w, h, Mu, Mp, a, nb, idx, gx, gy);
}

/*
 * Selected coefficients a_{us[k], ps[k]} over all n blocks, each an O(n) direct sum
 * (used to check the largest workloads, whose full coefficient set is too costly here).
 * Also returns the moments I (may be NULL).
 */
int oracle_coeffs_sampled_full(double W, double H, int64_t n, const double *x, const double *y,
                               const double *w, const double *h, int ns, const int *us, const int *ps,
                               double *a, double *I, double *R, double *Rabs)
{
    if (!(W > 0) || !(H > 0) || n < 0 || ns < 0) return -2;
    const int64_t CH = 8192;
    int64_t nch = (n + CH - 1) / CH;
    size_t np = (size_t)(nch > 0 ? nch : 1) * (size_t)(ns > 0 ? ns : 1);
    long double *part = (long double *)malloc(sizeof(long double) * np);
    long double *pabs = (long double *)malloc(sizeof(long double) * np);
    if (!part || !pabs) { free(part); free(pabs); return -1; }
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t c = 0; c < nch; ++c) {
        int64_t i0 = c * CH, i1 = (i0 + CH < n) ? i0 + CH : n;
        for (int k = 0; k < ns; ++k) {
            long double s = 0.0L, sa = 0.0L;
            for (int64_t i = i0; i < i1; ++i) {
                double Sx, Kx, Ty, Ly;
                if (us[k] == 0) Sx = w[i]; else edge_diffs(us[k], x[i], w[i], W, &Sx, &Kx);
                if (ps[k] == 0) Ty = h[i]; else edge_diffs(ps[k], y[i], h[i], H, &Ty, &Ly);
                s += (long double)Sx * (long double)Ty;
                sa += fabsl((long double)Sx * (long double)Ty);
            }
            part[(size_t)c * ns + k] = s;
            pabs[(size_t)c * ns + k] = sa;
        }
    }
    for (int k = 0; k < ns; ++k) {
        long double r = 0.0L, ra = 0.0L;
        for (int64_t c = 0; c < nch; ++c) {
            r += part[(size_t)c * ns + k];
            ra += pabs[(size_t)c * ns + k];
        }
        if (a) a[k] = (double)(coef_factor(us[k], ps[k], W, H) * r);
        if (I) I[k] = (double)(moment_factor(us[k], ps[k], W, H) * r);
        if (R) R[k] = (double)r;
        if (Rabs) Rabs[k] = (double)ra;
    }
    free(part);
    free(pabs);
    return 0;
}

/* Coefficients and moments only (the raw sums and their absolute counterparts are the
 * sampled-full call's). */
int oracle_coeffs_sampled(double W, double H, int64_t n, const double *x, const double *y,
                          const double *w, const double *h, int ns, const int *us, const int *ps,
                          double *a, double *I)
{
    return oracle_coeffs_sampled_full(W, H, n, x, y, w, h, ns, us, ps, a, I, NULL, NULL);
}

/*
 * Point values at (px[k], py[k]): psi (eq. psi) and the field xi = -grad psi (eq. ksi).
 * Any output pointer may be NULL.
 */
int oracle_point_field(double W, double H, int Mu, int Mp, const double *a, int64_t npts,
                       const double *px, const double *py, double *psi, double *xix, double *xiy)
{
    if (!(W > 0) || !(H > 0) || Mu < 1 || Mp < 1 || npts < 0) return -2;
    int fail = 0;
#pragma omp parallel
    {
        double *cu = (double *)malloc(sizeof(double) * (size_t)(2 * Mu + 2 * Mp));
        if (!cu) {
#pragma omp atomic write
            fail = 1;
        }
#pragma omp for schedule(dynamic, 4)
        for (int64_t k = 0; k < npts; ++k) {
            if (!cu) continue;
            double *su = cu + Mu, *cp = cu + 2 * Mu, *sp = cu + 2 * Mu + Mp;
            for (int u = 0; u < Mu; ++u) sincos_kpi(u, px[k], W, &su[u], &cu[u]);
            for (int p = 0; p < Mp; ++p) sincos_kpi(p, py[k], H, &sp[p], &cp[p]);
            long double ps = 0.0L, ex = 0.0L, ey = 0.0L;
            for (int u = 0; u < Mu; ++u) {
                const double *au = a + (size_t)u * Mp;
                long double zc = 0.0L, zs = 0.0L;
                for (int p = 0; p < Mp; ++p) {
                    zc += (long double)au[p] * cp[p];
                    zs += (long double)au[p] * ((double)p * ORACLE_PI / H) * sp[p];
                }
                ps += cu[u] * zc;
                ex += ((double)u * ORACLE_PI / W) * su[u] * zc;
                ey += cu[u] * zs;
            }
            if (psi) psi[k] = (double)ps;
            if (xix) xix[k] = (double)ex;
            if (xiy) xiy[k] = (double)ey;
        }
        free(cu);
    }
    return fail ? -1 : 0;
}

/* Block potentials N_i = iint_{block i} psi = sum_up a_up Xbar_iu Ybar_ip (E = 1/2 sum_i N_i). */
int oracle_block_potential(double W, double H, int64_t n, const double *x, const double *y,
                           const double *w, const double *h, int Mu, int Mp, const double *a,
                           double *N)
{
    if (!(W > 0) || !(H > 0) || Mu < 1 || Mp < 1 || n < 0) return -2;
    int fail = 0;
#pragma omp parallel
    {
        double *Xb = (double *)malloc(sizeof(double) * (size_t)(Mu + Mp));
        if (!Xb) {
#pragma omp atomic write
            fail = 1;
        }
#pragma omp for schedule(dynamic, 16)
        for (int64_t i = 0; i < n; ++i) {
            if (!Xb) continue;
            double *Yb = Xb + Mu;
            for (int u = 0; u < Mu; ++u) Xb[u] = edge_integral(u, x[i], w[i], W);
            for (int p = 0; p < Mp; ++p) Yb[p] = edge_integral(p, y[i], h[i], H);
            long double s = 0.0L;
            for (int u = 0; u < Mu; ++u) {
                const double *au = a + (size_t)u * Mp;
                long double z = 0.0L;
                for (int p = 0; p < Mp; ++p) z += (long double)au[p] * Yb[p];
                s += Xb[u] * z;
            }
            N[i] = (double)s;
        }
        free(Xb);
    }
    return fail ? -1 : 0;
}


/* ---------------------------------------------------------------------------------------------
 * 6. Bin scheme (Sec. III-D).  Bin arrays are row-major over (l, j): P[l*m + j].
 * ------------------------------------------------------------------------------------------- */

/* cos and sin of k (2s+1) pi / (2m), the argument reduced exactly modulo 4m first. */
static void bin_trig(long k, long s, long m, double *c, double *sn)
{
    long q = (k * (2 * s + 1)) % (4 * m);
    double phi = ORACLE_PI * (double)q / (2.0 * (double)m);
    *c = cos(phi);
    *sn = sin(phi);
}

/* The factor of the binned coefficient (u, p) in eqs. disa-a..d. */
static double bin_factor(long u, long p, double W, double H, long m)
{
    const double pi = ORACLE_PI;
    if (u == 0 && p == 0) return 0.0;
    if (u == 0) return 4.0 * H * H / ((double)p * p * p * pi * pi * pi * m) * sin(p * pi / (2.0 * m));
    if (p == 0) return 4.0 * W * W / ((double)u * u * u * pi * pi * pi * m) * sin(u * pi / (2.0 * m));
    return 16.0 * W * W * H * H / ((double)u * p * ((double)u * u * H * H + (double)p * p * W * W) *
                                   pi * pi * pi * pi) *
           sin(u * pi / (2.0 * m)) * sin(p * pi / (2.0 * m));
}

/* Bin densities: the overlap area of every block with every bin, over the bin area. */
int oracle_bin_density(double W, double H, int64_t n, const double *x, const double *y,
                       const double *w, const double *h, int m, double *P)
{
    if (m <= 0 || W <= 0.0 || H <= 0.0) return -1;
    const double wb = W / m, hb = H / m;
    long double *acc = (long double *)calloc((size_t)m * m, sizeof(long double));
    if (!acc) return -2;
    for (int64_t i = 0; i < n; ++i) {
        const double x0 = x[i] - w[i] / 2.0, x1 = x[i] + w[i] / 2.0;
        const double y0 = y[i] - h[i] / 2.0, y1 = y[i] + h[i] / 2.0;
        for (int l = 0; l < m; ++l) {
            const double ox = fmin(x1, (l + 1) * wb) - fmax(x0, l * wb);
            if (ox <= 0.0) continue;
            for (int j = 0; j < m; ++j) {
                const double oy = fmin(y1, (j + 1) * hb) - fmax(y0, j * hb);
                if (oy <= 0.0) continue;
                acc[(size_t)l * m + j] += (long double)(ox * oy);
            }
        }
    }
    for (size_t k = 0; k < (size_t)m * m; ++k) P[k] = (double)(acc[k] / ((long double)wb * hb));
    free(acc);
    return 0;
}

/* Binned coefficients a[u*Mp + p] (eqs. disa-a..d), u < Mu, p < Mp. */
int oracle_bin_coeffs(double W, double H, int m, const double *P, int Mu, int Mp, double *a)
{
    if (m <= 0 || Mu <= 0 || Mp <= 0) return -1;
    int st = 0;
#pragma omp parallel for schedule(dynamic)
    for (int u = 0; u < Mu; ++u) {
        for (int p = 0; p < Mp; ++p) {
            long double sum = 0.0L;
            for (int l = 0; l < m; ++l) {
                double cu, su;
                bin_trig(u, l, m, &cu, &su);
                for (int j = 0; j < m; ++j) {
                    double cp, sp;
                    bin_trig(p, j, m, &cp, &sp);
                    sum += (long double)P[(size_t)l * m + j] * cu * cp;
                }
            }
            a[(size_t)u * Mp + p] = (double)(bin_factor(u, p, W, H, m) * sum);
        }
    }
    return st;
}

/* Potential and field at the bin centres (eqs. dis-psi1, dis-ksi); NULL outputs are skipped. */
int oracle_bin_field(double W, double H, int m, int Mu, int Mp, const double *a, double *psi,
                     double *xix, double *xiy)
{
    if (m <= 0 || Mu <= 0 || Mp <= 0) return -1;
    const double pi = ORACLE_PI;
    int fail = 0;
#pragma omp parallel for schedule(dynamic)
    for (int l = 0; l < m; ++l) {
        double *cu = (double *)malloc(sizeof(double) * (size_t)(2 * Mu + 2 * Mp));
        if (!cu) {
#pragma omp atomic write
            fail = 1;
            continue;
        }
        double *su = cu + Mu, *cp = su + Mu, *sp = cp + Mp;
        for (int u = 0; u < Mu; ++u) bin_trig(u, l, m, &cu[u], &su[u]);
        for (int j = 0; j < m; ++j) {
            for (int p = 0; p < Mp; ++p) bin_trig(p, j, m, &cp[p], &sp[p]);
            long double e = 0.0L, ex = 0.0L, ey = 0.0L;
            for (int u = 0; u < Mu; ++u)
                for (int p = 0; p < Mp; ++p) {
                    const double apu = a[(size_t)u * Mp + p];
                    e += (long double)apu * cu[u] * cp[p];
                    ex += (long double)((double)u * pi / W) * apu * su[u] * cp[p];
                    ey += (long double)((double)p * pi / H) * apu * cu[u] * sp[p];
                }
            if (psi) psi[(size_t)l * m + j] = (double)e;
            if (xix) xix[(size_t)l * m + j] = (double)ex;
            if (xiy) xiy[(size_t)l * m + j] = (double)ey;
        }
        free(cu);
    }
    return fail ? -2 : 0;
}

/* Selected bin densities P[ls[k], js[k]] (the same sums as oracle_bin_density, for large grids). */
int oracle_bin_density_at(double W, double H, int64_t n, const double *x, const double *y,
                          const double *w, const double *h, int m, int64_t count, const int *ls,
                          const int *js, double *out)
{
    if (m <= 0 || W <= 0.0 || H <= 0.0) return -1;
    const double wb = W / m, hb = H / m;
#pragma omp parallel for schedule(dynamic)
    for (int64_t k = 0; k < count; ++k) {
        const int l = ls[k], j = js[k];
        long double acc = 0.0L;
        for (int64_t i = 0; i < n; ++i) {
            const double ox = fmin(x[i] + w[i] / 2.0, (l + 1) * wb) - fmax(x[i] - w[i] / 2.0, l * wb);
            const double oy = fmin(y[i] + h[i] / 2.0, (j + 1) * hb) - fmax(y[i] - h[i] / 2.0, j * hb);
            if (ox > 0.0 && oy > 0.0) acc += (long double)(ox * oy);
        }
        out[k] = (double)(acc / ((long double)wb * hb));
    }
    return 0;
}

/* Selected binned coefficients a[us[k], ps[k]] (the same sums as oracle_bin_coeffs). */
int oracle_bin_coeffs_at(double W, double H, int m, const double *P, int64_t count, const int *us,
                         const int *ps, double *out)
{
    if (m <= 0) return -1;
#pragma omp parallel for schedule(dynamic)
    for (int64_t k = 0; k < count; ++k) {
        const int u = us[k], p = ps[k];
        long double sum = 0.0L;
        for (int l = 0; l < m; ++l) {
            double cu, su;
            bin_trig(u, l, m, &cu, &su);
            for (int j = 0; j < m; ++j) {
                double cp, sp;
                bin_trig(p, j, m, &cp, &sp);
                sum += (long double)P[(size_t)l * m + j] * cu * cp;
            }
        }
        out[k] = (double)(bin_factor(u, p, W, H, m) * sum);
    }
    return 0;
}

/* Block values from bin values (the last step of the scheme): for each block, the sum over the
 * bins it overlaps of the overlap area times the bin value; the field sums carry a minus sign so
 * that they approximate the gradient dE/dx_i, dE/dy_i.  A NULL field skips its output. */
int oracle_bin_interp(double W, double H, int64_t n, const double *x, const double *y,
                      const double *w, const double *h, int m, const double *psi, const double *xix,
                      const double *xiy, double *N, double *gx, double *gy)
{
    if (m <= 0 || W <= 0.0 || H <= 0.0) return -1;
    const double wb = W / m, hb = H / m;
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < n; ++i) {
        const double x0 = x[i] - w[i] / 2.0, x1 = x[i] + w[i] / 2.0;
        const double y0 = y[i] - h[i] / 2.0, y1 = y[i] + h[i] / 2.0;
        long double sp = 0.0L, sx = 0.0L, sy = 0.0L;
        for (int l = 0; l < m; ++l) {
            const double ox = fmin(x1, (l + 1) * wb) - fmax(x0, l * wb);
            if (ox <= 0.0) continue;
            for (int j = 0; j < m; ++j) {
                const double oy = fmin(y1, (j + 1) * hb) - fmax(y0, j * hb);
                if (oy <= 0.0) continue;
                const long double area = (long double)ox * oy;
                const size_t b = (size_t)l * m + j;
                if (psi) sp += area * psi[b];
                if (xix) sx += area * xix[b];
                if (xiy) sy += area * xiy[b];
            }
        }
        if (psi) N[i] = (double)sp;
        if (xix) gx[i] = (double)-sx;
        if (xiy) gy[i] = (double)-sy;
    }
    return 0;
}
