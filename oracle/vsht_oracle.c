/*
 * vsht_oracle.c -- plain, slow CPU reference for the forward and adjoint
 * vector spherical harmonic transforms (FaVeST, Le Gia, Li and Wang).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may link, load or
 * call this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, table or helper with the HIP
 * library.
 *
 * What it computes (in IEEE binary64, built with -ffp-contract=off; only the
 * Legendre recurrence runs in the x87 extended type, for its exponent range):
 *   - scalar spherical harmonics Y_{l,m} of Section 3 (4pi-orthonormal, with
 *     the Condon-Shortley phase; negative orders use the conjugate relation
 *     Y_{l,-m} = (-1)^m conj(Y_{l,m}), the orthonormal reading of the
 *     negative-order definition in Section 3);
 *   - the vector spherical harmonics Y^div and Y^curl of Definition 3.1,
 *     assembled exactly as the paper writes them: the B and D coefficients of
 *     eq. (Blm1)/(Blm2), the nine Clebsch-Gordan closed forms of
 *     eq. (ninecoeff), the constants c_l, d_l of eq. (cl,dl,betal) and the
 *     Cartesian form eq. (vsh2);
 *   - the forward transform of Definition 4.1, eq. (fwdvsht2):
 *         a_{l,m} = sum_k w_k Y^div_{l,m}(x_k)^* T_k ,  b likewise with Y^curl;
 *   - the adjoint transform of Definition 4.2, eq. (SLvec):
 *         T(x_i) = sum_{l=1}^{L} sum_{|m|<=l} a_{l,m} Y^div_{l,m}(x_i) + b_{l,m} Y^curl_{l,m}(x_i).
 * These are direct O(N L^2) sums of the definitions; the paper's Theorems 1
 * and 2 state that its fast method reaches exactly these sums.
 *
 * Layouts (shared with the library's public interface, nothing else):
 *   points   xyz[k*3 + c]                  unit vectors, row-major (n,3)
 *   field    T[(k*3 + c)*2 + {0,1}]         complex (n,3) as interleaved re/im
 *   coeffs   a[(l*l + l + m - 1)*2 + {0,1}]  1 <= l <= L, -l <= m <= l
 *   scalar   Y[(l*l + l + m)*2 + {0,1}]      0 <= l <= Lmax
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

static const double ORC_PI = 3.14159265358979323846264338327950288;
static const long double ORC_PIL = 3.14159265358979323846264338327950288L;

/* ---------------------------------------------------------------------- */
/* Point geometry: z = cos(theta), s = sin(theta) >= 0, phi = longitude.   */
/* At the poles (s == 0) phi is taken as 0; every Y_{l,m} with m != 0      */
/* vanishes there, so the choice does not matter.                          */
/* ---------------------------------------------------------------------- */
static void point_geometry(const double *x, double *z, double *s, double *phi)
{
    *z = x[2];
    *s = sqrt(x[0] * x[0] + x[1] * x[1]);
    *phi = (*s > 0.0) ? atan2(x[1], x[0]) : 0.0;
}

/* ---------------------------------------------------------------------- */
/* Normalised associated Legendre functions (Section 3):                   */
/*   Pbar_{l,m}(z) = sqrt((2l+1)/(4pi) (l-m)!/(l+m)!) P_l^m(z),  m >= 0,   */
/* with the Condon-Shortley factor (-1)^m inside P_l^m.  Textbook           */
/* three-term recurrence in l at fixed m, started from the closed form     */
/*   Pbar_{m,m} = (-1)^m sqrt((2m+1)/(4pi) prod_{k=1}^{m} (2k-1)/(2k)) s^m */
/*   Pbar_{m+1,m} = sqrt(2m+3) z Pbar_{m,m}                                 */
/*   Pbar_{l,m} = A (z Pbar_{l-1,m} - B Pbar_{l-2,m}),                      */
/*     A = sqrt((4l^2-1)/(l^2-m^2)),  B = sqrt(((l-1)^2-m^2)/(4(l-1)^2-1)). */
/* The seed Pbar_{m,m} = O(s^m) leaves binary64's range near the poles     */
/* long before the functions it starts become negligible (at L ~ 2000 a     */
/* seed of 1e-400 grows to O(1) by l = L), so the recurrence runs in the   */
/* x87 extended type (15-bit exponent, down to 1e-4951; a seed below that   */
/* cannot grow past ~1e-4400 within l <= 4096) and each value is rounded   */
/* to binary64 once, when stored.                                           */
/* Table P[m][l] stored as P[m*(Lmax+1) + l] (entries l < m unused).        */
/* ---------------------------------------------------------------------- */
typedef long double xreal;

static xreal legendre_step(int l, int m, xreal z, xreal p1, xreal p2)
{
    const xreal L = l, M = m;
    xreal A = sqrtl((4.0L * L * L - 1.0L) / (L * L - M * M));
    xreal B = sqrtl(((L - 1.0L) * (L - 1.0L) - M * M) / (4.0L * (L - 1.0L) * (L - 1.0L) - 1.0L));
    return A * (z * p1 - B * p2);
}

static void legendre_table(int Lmax, double z, double s, double *P)
{
    const int ld = Lmax + 1;
    const xreal zx = z, sx = s;
    xreal pmm = sqrtl(1.0L / (4.0L * ORC_PIL));
    for (int m = 0; m <= Lmax; ++m) {
        if (m > 0)
            pmm = -pmm * sx * sqrtl((2.0L * m + 1.0L) / (2.0L * m));
        double *col = P + (size_t)m * ld;
        col[m] = (double)pmm;
        xreal p2 = pmm, p1 = sqrtl(2.0L * m + 3.0L) * zx * pmm;
        if (m + 1 <= Lmax)
            col[m + 1] = (double)p1;
        for (int l = m + 2; l <= Lmax; ++l) {
            xreal cur = legendre_step(l, m, zx, p1, p2);
            col[l] = (double)cur;
            p2 = p1;
            p1 = cur;
        }
    }
}

/* Y_{l,m} from the Legendre table and the longitude phi (Section 3). */
static cplx ylm_from_table(int Lmax, const double *P, int l, int m, double phi)
{
    if (l < 0 || l > Lmax || m > l || -m > l)
        return 0.0;
    int am = m < 0 ? -m : m;
    double p = P[(size_t)am * (Lmax + 1) + l];
    cplx e = cos(m * phi) + I * sin(m * phi);
    if (m < 0 && (am & 1))
        p = -p; /* Y_{l,-|m|} = (-1)^{|m|} conj(Y_{l,|m|}) */
    return p * e;
}

/* ---------------------------------------------------------------------- */
/* Vector spherical harmonics from the nine neighbouring scalar harmonics  */
/* Y_{l+dl, m+dm}, dl, dm in {-1,0,1} (Ynb[dl+1][dm+1], zero outside the    */
/* range 0 <= l', |m'| <= l').  Every factor is the paper's:                 */
/*   c_l, d_l                      eq. (cl,dl,betal)                         */
/*   nine CG closed forms          eq. (ninecoeff)                           */
/*   B_{q,l,m}, D_{q,l,m}          eq. (Blm1), eq. (Blm2)                    */
/*   Cartesian components          eq. (vsh2)                                */
/* A term is only formed when its scalar harmonic exists, so no square root */
/* of a negative number is ever taken.                                      */
/* ---------------------------------------------------------------------- */
static void vsh_from_neighbours(int l, int m, cplx Ynb[3][3], cplx ydiv[3], cplx ycurl[3])
{
    const double L = (double)l, M = (double)m;
    const double cl = sqrt((L + 1.0) / (2.0 * L + 1.0));
    const double dl = sqrt(L / (2.0 * L + 1.0));
    const double r2 = sqrt(2.0);
    cplx Bp = 0.0, B0 = 0.0, Bm = 0.0;

    /* B_{+1,l,m} = c_l C^{l,m}_{l-1,m-1,1,1} Y_{l-1,m-1} + d_l C^{l,m}_{l+1,m-1,1,1} Y_{l+1,m-1} */
    if (Ynb[0][0] != 0.0)
        Bp += cl * sqrt((L + M) * (L + M - 1.0) / ((2.0 * L) * (2.0 * L - 1.0))) * Ynb[0][0];
    if (Ynb[2][0] != 0.0)
        Bp += dl * sqrt((L - M + 1.0) * (L - M + 2.0) / ((2.0 * L + 2.0) * (2.0 * L + 3.0))) * Ynb[2][0];
    /* B_{0,l,m} = c_l C^{l,m}_{l-1,m,1,0} Y_{l-1,m} + d_l C^{l,m}_{l+1,m,1,0} Y_{l+1,m} */
    if (Ynb[0][1] != 0.0)
        B0 += cl * sqrt((L + M) * (L - M) / (L * (2.0 * L - 1.0))) * Ynb[0][1];
    if (Ynb[2][1] != 0.0)
        B0 += dl * -sqrt((L - M + 1.0) * (L + M + 1.0) / ((2.0 * L + 3.0) * (L + 1.0))) * Ynb[2][1];
    /* B_{-1,l,m} = c_l C^{l,m}_{l-1,m+1,1,-1} Y_{l-1,m+1} + d_l C^{l,m}_{l+1,m+1,1,-1} Y_{l+1,m+1} */
    if (Ynb[0][2] != 0.0)
        Bm += cl * sqrt((L - M) * (L - M - 1.0) / ((2.0 * L) * (2.0 * L - 1.0))) * Ynb[0][2];
    if (Ynb[2][2] != 0.0)
        Bm += dl * sqrt((L + M + 1.0) * (L + M + 2.0) / ((2.0 * L + 3.0) * (2.0 * L + 2.0))) * Ynb[2][2];

    /* D_{+1} = i C^{l,m}_{l,m-1,1,1} Y_{l,m-1}, D_0 = i C^{l,m}_{l,m,1,0} Y_{l,m},
       D_{-1} = i C^{l,m}_{l,m+1,1,-1} Y_{l,m+1} */
    cplx Dp = 0.0, D0 = 0.0, Dm = 0.0;
    if (Ynb[1][0] != 0.0)
        Dp = I * -sqrt((L + M) * (L - M + 1.0) / (L * (2.0 * L + 2.0))) * Ynb[1][0];
    D0 = I * (M / sqrt(L * (L + 1.0))) * Ynb[1][1];
    if (Ynb[1][2] != 0.0)
        Dm = I * sqrt((L + M + 1.0) * (L - M) / (L * (2.0 * L + 2.0))) * Ynb[1][2];

    /* eq. (vsh2) */
    ydiv[0] = -(Bp - Bm) / r2;
    ydiv[1] = -I * (Bp + Bm) / r2;
    ydiv[2] = B0;
    ycurl[0] = -(Dp - Dm) / r2;
    ycurl[1] = -I * (Dp + Dm) / r2;
    ycurl[2] = D0;
}

/* Fill the 3x3 neighbourhood of (l,m) from a full table of Y_{l',m'}. */
static void neighbours_from_full(int Lmax, const cplx *Y, int l, int m, cplx Ynb[3][3])
{
    for (int a = 0; a < 3; ++a)
        for (int c = 0; c < 3; ++c) {
            int lp = l + a - 1, mp = m + c - 1;
            Ynb[a][c] = (lp >= 0 && lp <= Lmax && mp <= lp && -mp <= lp)
                            ? Y[(size_t)lp * lp + lp + mp] : 0.0;
        }
}

/* All Y_{l,m}, 0 <= l <= Lmax, at one point into Y[l*l+l+m]; P is scratch. */
static void ylm_all_point(int Lmax, const double *x, double *P, cplx *Y)
{
    double z, s, phi;
    point_geometry(x, &z, &s, &phi);
    legendre_table(Lmax, z, s, P);
    for (int l = 0; l <= Lmax; ++l)
        for (int m = -l; m <= l; ++m)
            Y[(size_t)l * l + l + m] = ylm_from_table(Lmax, P, l, m, phi);
}

/* ====================================================================== */
/* Exported entry points (ctypes).                                         */
/* ====================================================================== */

int vo_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Scalar harmonics Y_{l,m}, 0 <= l <= Lmax, at n points: out[(k*(Lmax+1)^2 + l*l+l+m)*2]. */
void vo_sph_harm(int Lmax, int64_t n, const double *xyz, double *out)
{
    const size_t nY = (size_t)(Lmax + 1) * (Lmax + 1);
#pragma omp parallel
    {
        double *P = malloc(sizeof(double) * (size_t)(Lmax + 1) * (Lmax + 1));
#pragma omp for schedule(static)
        for (int64_t k = 0; k < n; ++k)
            ylm_all_point(Lmax, xyz + 3 * k, P, (cplx *)out + (size_t)k * nY);
        free(P);
    }
}

/* Vector harmonics at n points:
 * div[((k*K + j)*3 + c)*2], curl likewise, j = l*l+l+m-1, K = L(L+2). */
void vo_vsh(int L, int64_t n, const double *xyz, double *div, double *curl)
{
    const int Lmax = L + 1;
    const size_t nY = (size_t)(Lmax + 1) * (Lmax + 1);
    const size_t K = (size_t)L * (L + 2);
#pragma omp parallel
    {
        double *P = malloc(sizeof(double) * nY);
        cplx *Y = malloc(sizeof(cplx) * nY);
#pragma omp for schedule(static)
        for (int64_t k = 0; k < n; ++k) {
            ylm_all_point(Lmax, xyz + 3 * k, P, Y);
            for (int l = 1; l <= L; ++l)
                for (int m = -l; m <= l; ++m) {
                    cplx nb[3][3], yd[3], yc[3];
                    neighbours_from_full(Lmax, Y, l, m, nb);
                    vsh_from_neighbours(l, m, nb, yd, yc);
                    size_t j = (size_t)l * l + l + m - 1;
                    for (int c = 0; c < 3; ++c) {
                        ((cplx *)div)[((size_t)k * K + j) * 3 + c] = yd[c];
                        ((cplx *)curl)[((size_t)k * K + j) * 3 + c] = yc[c];
                    }
                }
        }
        free(P);
        free(Y);
    }
}

/* Forward transform, eq. (fwdvsht2), all coefficients.
 * The points are split into a fixed number of contiguous blocks; each block's
 * partial sum runs over its points in order and the blocks are added in order,
 * so the result does not depend on the thread count. */
void vo_forward(int L, int64_t n, const double *xyz, const double *w, const double *T,
                double *a_out, double *b_out)
{
    const int Lmax = L + 1;
    const size_t nY = (size_t)(Lmax + 1) * (Lmax + 1);
    const size_t K = (size_t)L * (L + 2);
    int64_t nblk = 64;
    while (nblk > 1 && (double)nblk * 2.0 * K * sizeof(cplx) > 2.0e9)
        nblk /= 2;
    if (nblk > n)
        nblk = n > 0 ? n : 1;
    cplx *part = calloc((size_t)nblk * 2 * K, sizeof(cplx));
    const cplx *Tc = (const cplx *)T;
#pragma omp parallel
    {
        double *P = malloc(sizeof(double) * nY);
        cplx *Y = malloc(sizeof(cplx) * nY);
#pragma omp for schedule(dynamic, 1)
        for (int64_t blk = 0; blk < nblk; ++blk) {
            int64_t k0 = n * blk / nblk, k1 = n * (blk + 1) / nblk;
            cplx *pa = part + (size_t)blk * 2 * K, *pb = pa + K;
            for (int64_t k = k0; k < k1; ++k) {
                ylm_all_point(Lmax, xyz + 3 * k, P, Y);
                const cplx *Tk = Tc + 3 * k;
                for (int l = 1; l <= L; ++l)
                    for (int m = -l; m <= l; ++m) {
                        cplx nb[3][3], yd[3], yc[3];
                        neighbours_from_full(Lmax, Y, l, m, nb);
                        vsh_from_neighbours(l, m, nb, yd, yc);
                        cplx sa = 0.0, sb = 0.0;
                        for (int c = 0; c < 3; ++c) {
                            sa += conj(yd[c]) * Tk[c];
                            sb += conj(yc[c]) * Tk[c];
                        }
                        size_t j = (size_t)l * l + l + m - 1;
                        pa[j] += w[k] * sa;
                        pb[j] += w[k] * sb;
                    }
            }
        }
        free(P);
        free(Y);
    }
    cplx *a = (cplx *)a_out, *b = (cplx *)b_out;
    for (size_t j = 0; j < K; ++j) {
        cplx sa = 0.0, sb = 0.0;
        for (int64_t blk = 0; blk < nblk; ++blk) {
            sa += part[(size_t)blk * 2 * K + j];
            sb += part[(size_t)blk * 2 * K + K + j];
        }
        a[j] = sa;
        b[j] = sb;
    }
    free(part);
}

/* Adjoint transform, eq. (SLvec), at every given point. */
void vo_adjoint(int L, const double *a_in, const double *b_in, int64_t n, const double *xyz,
                double *T_out)
{
    const int Lmax = L + 1;
    const size_t nY = (size_t)(Lmax + 1) * (Lmax + 1);
    const cplx *a = (const cplx *)a_in, *b = (const cplx *)b_in;
    cplx *T = (cplx *)T_out;
#pragma omp parallel
    {
        double *P = malloc(sizeof(double) * nY);
        cplx *Y = malloc(sizeof(cplx) * nY);
#pragma omp for schedule(dynamic, 1)
        for (int64_t k = 0; k < n; ++k) {
            ylm_all_point(Lmax, xyz + 3 * k, P, Y);
            cplx acc[3] = {0.0, 0.0, 0.0};
            for (int l = 1; l <= L; ++l)
                for (int m = -l; m <= l; ++m) {
                    cplx nb[3][3], yd[3], yc[3];
                    neighbours_from_full(Lmax, Y, l, m, nb);
                    vsh_from_neighbours(l, m, nb, yd, yc);
                    size_t j = (size_t)l * l + l + m - 1;
                    for (int c = 0; c < 3; ++c)
                        acc[c] += a[j] * yd[c] + b[j] * yc[c];
                }
            for (int c = 0; c < 3; ++c)
                T[3 * k + c] = acc[c];
        }
        free(P);
        free(Y);
    }
}

/* ---------------------------------------------------------------------- */
/* Forward transform for a chosen subset of coefficients (full point set). */
/* Same sum as vo_forward, coefficient by coefficient.  The Legendre values */
/* depend on a point only through z, so they are computed once per distinct */
/* z value (exact equality) and reused for every point with that z; the sum */
/* itself still visits every point in input order.                          */
/* ---------------------------------------------------------------------- */
typedef struct { double z; int64_t k; } zkey;

static int cmp_zkey(const void *p, const void *q)
{
    double a = ((const zkey *)p)->z, b = ((const zkey *)q)->z;
    if (a < b) return -1;
    if (a > b) return 1;
    int64_t i = ((const zkey *)p)->k, j = ((const zkey *)q)->k;
    return (i > j) - (i < j);
}

/* Pbar_{l,am}(z) for l = lo..hi (hi <= Lmax) by the same recurrence as
 * legendre_table (extended type), restricted to one order; out[l - lo], zero
 * for l < am. */
static void legendre_column(int am, int lo, int hi, double z, double s, double *out)
{
    const xreal zx = z, sx = s;
    xreal pmm = sqrtl(1.0L / (4.0L * ORC_PIL));
    for (int m = 1; m <= am; ++m)
        pmm = -pmm * sx * sqrtl((2.0L * m + 1.0L) / (2.0L * m));
    xreal p2 = 0.0L, p1 = pmm; /* Pbar_{l-2}, Pbar_{l-1} once l > am + 1 */
    for (int l = am; l <= hi; ++l) {
        xreal cur;
        if (l == am)
            cur = pmm;
        else if (l == am + 1)
            cur = sqrtl(2.0L * am + 3.0L) * zx * pmm;
        else
            cur = legendre_step(l, am, zx, p1, p2);
        if (l > am) { p2 = p1; p1 = cur; }
        if (l >= lo)
            out[l - lo] = (double)cur;
    }
    for (int l = lo; l <= hi && l < am; ++l)
        out[l - lo] = 0.0;
}

void vo_forward_subset(int L, int64_t n, const double *xyz, const double *w, const double *T,
                       int64_t ncoef, const int64_t *coef_index, double *a_out, double *b_out)
{
    (void)L; /* the degree of each coefficient is read from its index */
    const cplx *Tc = (const cplx *)T;
    /* distinct z values */
    zkey *keys = malloc(sizeof(zkey) * (size_t)n);
    for (int64_t k = 0; k < n; ++k) { keys[k].z = xyz[3 * k + 2]; keys[k].k = k; }
    qsort(keys, (size_t)n, sizeof(zkey), cmp_zkey);
    int64_t *zid = malloc(sizeof(int64_t) * (size_t)n);
    double *zval = malloc(sizeof(double) * (size_t)n);
    int64_t nz = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (i == 0 || keys[i].z != keys[i - 1].z)
            zval[nz++] = keys[i].z;
        zid[keys[i].k] = nz - 1;
    }
    free(keys);
    double *phi = malloc(sizeof(double) * (size_t)n);
    for (int64_t k = 0; k < n; ++k) {
        double z, s;
        point_geometry(xyz + 3 * k, &z, &s, phi + k);
    }
    cplx *a = (cplx *)a_out, *b = (cplx *)b_out;
#pragma omp parallel
    {
        /* memo[zi][dl][dm] = Pbar_{l+dl, |m+dm|}(z_zi) with the sign rule folded in later */
        double *memo = malloc(sizeof(double) * (size_t)nz * 9);
        double col[3];
#pragma omp for schedule(dynamic, 1)
        for (int64_t c = 0; c < ncoef; ++c) {
            int64_t j = coef_index[c];
            /* j = l*l + l + m - 1 with |m| <= l  <=>  l*l - 1 <= j <= (l+1)*(l+1) - 2 */
            int l = (int)floor(sqrt((double)(j + 1)));
            while ((int64_t)l * l - 1 > j) --l;
            while ((int64_t)(l + 1) * (l + 1) - 1 <= j) ++l;
            int m = (int)(j - ((int64_t)l * l + l - 1));
            for (int64_t zi = 0; zi < nz; ++zi) {
                double z = zval[zi];
                double s = sqrt((1.0 - z) * (1.0 + z));
                for (int dm = -1; dm <= 1; ++dm) {
                    int am = abs(m + dm);
                    legendre_column(am, l - 1, l + 1, z, s, col);
                    for (int dl = -1; dl <= 1; ++dl)
                        memo[(size_t)zi * 9 + (dl + 1) * 3 + (dm + 1)] = col[dl + 1];
                }
            }
            cplx sa = 0.0, sb = 0.0;
            for (int64_t k = 0; k < n; ++k) {
                cplx nb[3][3], yd[3], yc[3], e[3];
                const double *mk = memo + (size_t)zid[k] * 9;
                for (int dm = -1; dm <= 1; ++dm)
                    e[dm + 1] = cos((m + dm) * phi[k]) + I * sin((m + dm) * phi[k]);
                for (int dl = -1; dl <= 1; ++dl)
                    for (int dm = -1; dm <= 1; ++dm) {
                        int lp = l + dl, mp = m + dm, am = abs(mp);
                        if (lp < 0 || am > lp) { nb[dl + 1][dm + 1] = 0.0; continue; }
                        double p = mk[(dl + 1) * 3 + (dm + 1)];
                        if (mp < 0 && (am & 1)) p = -p;
                        nb[dl + 1][dm + 1] = p * e[dm + 1];
                    }
                vsh_from_neighbours(l, m, nb, yd, yc);
                cplx ta = 0.0, tb = 0.0;
                for (int cc = 0; cc < 3; ++cc) {
                    ta += conj(yd[cc]) * Tc[3 * k + cc];
                    tb += conj(yc[cc]) * Tc[3 * k + cc];
                }
                sa += w[k] * ta;
                sb += w[k] * tb;
            }
            a[c] = sa;
            b[c] = sb;
        }
        free(memo);
    }
    free(zid);
    free(zval);
    free(phi);
}
