/*
 * cholinv_oracle_q15.c -- integer CPU oracle of the fixed-point form of the
 * proposed inversion (Cholesky, Section II eqs. (3)-(4); Section IV.A
 * back-substitution), for complex Hermitian matrices in Q15.
 *
 * TEST INFRASTRUCTURE ONLY (built into the oracle library; loaded only by the
 * tests, the smoke check and the benchmark's CPU leg).  Shares nothing with
 * the GPU library.
 *
 * The paper evaluates its method by fixed-point simulation but states no
 * format.  This file fixes one (the reading is listed with the design notes):
 *   - input entries q_ij (int16 re, im) stand for a_ij = q_ij / 2^15; only
 *     the upper triangle is read and the imaginary part of a_ii is ignored;
 *   - R is held in Q15 (int16 range), every sum of products in int64 with 30
 *     fractional bits;
 *   - r_ii = floor(sqrt(sum)) exactly (a Q30 radicand gives a Q15 root),
 *     r_ij = sum / r_ii by integer division rounded to nearest, halves away
 *     from zero; results beyond +-32767 saturate and are counted;
 *   - X is built in int64 as Y = X 2^F with one exponent per matrix,
 *     F = 2 floor(log2 min_i r_ii) - ceil(log2 n) (so that |x| <= n / r_min^2
 *     lands below 2^30); Y parts saturate at +-(2^40 - 1), counted;
 *   - the result is rounded to int16 mantissas with one exponent per matrix:
 *     x_ij = X_ij 2^xexp, the smallest shift that fits, mirrored as
 *     x_ji = conj(x_ij).
 * A radicand <= 0 stops the factorisation: info = 1-based row, X = 0.
 *
 * The comparison methods of Section III in the same format (or_inv_q15_cmp):
 * the same factor R, the same Y = X 2^F, exponent search and output; only the
 * route from R to Y differs.  Both hold an intermediate (the forward solution
 * b of III.A, M = R^{-1} of III.B) as W = (.) 2^G in int64 with
 * G = floor(log2 min r_ii) + 13 - ceil(ceil(log2 n) / 2), saturating at
 * +-(2^29 - 1), so that every sum of products of two such values (at most 32
 * per part for n <= 16) stays below 2^63:
 *   III.A (eq. 15) column i = n-1..0: forward R^* b = e_i for rows j >= i,
 *     w_i = 2^(G+15) / r_ii, w_j = -(sum_{k=i}^{j-1} conj(r_kj) w_k) / r_jj;
 *     then backward R x = b for rows j = i..0,
 *     y_ji = (w_j 2^(F+15-G) - sum_{k>j} r_jk yh_ki) / r_jj, yh_ki = y_ki for
 *     k <= i and conj(y_ik) from the columns already solved;
 *   III.B (eqs. 17-19): M = R^{-1} column by column, rows j = i..0,
 *     w_ii = 2^(G+15) / r_ii, w_ji = -(sum_{k=j+1}^{i} r_jk w_ki) / r_jj; then
 *     y_ij = (sum_{k>=j} w_ik conj(w_jk)) / 2^(2G-F) for i <= j.
 * Every division is the same rounded integer division; the terms known to be
 * zero are not summed (integer sums are exact, so this changes no result).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* floor(sqrt(v)) for v >= 0, binary digit-by-digit (restoring) method */
static int64_t q_isqrt(int64_t v)
{
    int64_t rem = v, root = 0, bit = (int64_t)1 << 62;
    while (bit > rem) bit >>= 2;
    while (bit) {
        if (rem >= root + bit) {
            rem -= root + bit;
            root = (root >> 1) + bit;
        } else {
            root >>= 1;
        }
        bit >>= 2;
    }
    return root;
}

/* num / den rounded to nearest, halves away from zero (den > 0): the
 * quotient of |num| goes up by one when twice the remainder reaches den */
static int64_t q_rdiv(int64_t num, int64_t den)
{
    const int64_t m = num < 0 ? -num : num;
    int64_t q = m / den;
    if (2 * (m - q * den) >= den) ++q;
    return num < 0 ? -q : q;
}

static int64_t q_clip(int64_t v, int64_t lim, int32_t* sat)
{
    if (v > lim) { ++*sat; return lim; }
    if (v < -lim) { ++*sat; return -lim; }
    return v;
}

#define Q15_MAX 32767
#define Y_LIM (((int64_t)1 << 40) - 1)
#define W_LIM (((int64_t)1 << 29) - 1)

/* eqs. (3)-(4), row by row, on the upper triangle of the n x n int16 (re, im)
 * matrix a: R into rr, ri (n x n, upper part).  Returns 0 or the 1-based row
 * whose radicand is <= 0. */
static int q15_factor(int n, const int16_t* a, int64_t* rr, int64_t* ri, int32_t* sat)
{
#define A_RE(i, j) ((int64_t)a[2 * ((size_t)(i) * n + (j))])
#define A_IM(i, j) ((int64_t)a[2 * ((size_t)(i) * n + (j)) + 1])
#define IX(i, j) ((size_t)(i) * n + (j))
    for (int i = 0; i < n; ++i) {
        int64_t acc = A_RE(i, i) * 32768;                      /* Q30 */
        for (int k = 0; k < i; ++k)
            acc -= rr[IX(k, i)] * rr[IX(k, i)] + ri[IX(k, i)] * ri[IX(k, i)];
        if (acc <= 0) return i + 1;
        const int64_t d = q_isqrt(acc);                        /* Q15, >= 1 */
        rr[IX(i, i)] = d;
        ri[IX(i, i)] = 0;
        for (int j = i + 1; j < n; ++j) {
            int64_t sr = A_RE(i, j) * 32768, si = A_IM(i, j) * 32768;
            for (int k = 0; k < i; ++k) {                      /* conj(r_ki) r_kj */
                sr -= rr[IX(k, i)] * rr[IX(k, j)] + ri[IX(k, i)] * ri[IX(k, j)];
                si -= rr[IX(k, i)] * ri[IX(k, j)] - ri[IX(k, i)] * rr[IX(k, j)];
            }
            rr[IX(i, j)] = q_clip(q_rdiv(sr, d), Q15_MAX, sat);
            ri[IX(i, j)] = q_clip(q_rdiv(si, d), Q15_MAX, sat);
        }
    }
    return 0;
#undef A_RE
#undef A_IM
#undef IX
}

/* floor(log2 min r_ii): 2^b <= min r_ii */
static int q15_log2_rmin(int n, const int64_t* rr)
{
    int64_t rmin = Q15_MAX;
    for (int i = 0; i < n; ++i)
        if (rr[(size_t)i * n + i] < rmin) rmin = rr[(size_t)i * n + i];
    int b = 0;
    while ((rmin >> (b + 1)) > 0) ++b;
    return b;
}

static int q15_ceil_log2(int n)
{
    int lg = 0;
    while ((1 << lg) < n) ++lg;
    return lg;
}

/* int16 mantissas of Y = X 2^F (upper half) with one exponent, mirrored */
static void q15_emit(int n, const int64_t* yr, const int64_t* yi, int F, int16_t* x,
                     int32_t* xexp)
{
#define IX(i, j) ((size_t)(i) * n + (j))
    int64_t m = 0;
    for (int i = 0; i < n; ++i)
        for (int j = i; j < n; ++j) {
            const int64_t ar = yr[IX(i, j)] < 0 ? -yr[IX(i, j)] : yr[IX(i, j)];
            const int64_t ai = yi[IX(i, j)] < 0 ? -yi[IX(i, j)] : yi[IX(i, j)];
            if (ar > m) m = ar;
            if (ai > m) m = ai;
        }
    int s = 0;
    while (q_rdiv(m, (int64_t)1 << s) > Q15_MAX) ++s;
    for (int i = 0; i < n; ++i)
        for (int j = i; j < n; ++j) {
            const int16_t xr = (int16_t)q_rdiv(yr[IX(i, j)], (int64_t)1 << s);
            const int16_t xi = (int16_t)q_rdiv(yi[IX(i, j)], (int64_t)1 << s);
            x[2 * IX(i, j)] = xr;
            x[2 * IX(i, j) + 1] = xi;
            x[2 * IX(j, i)] = xr;
            x[2 * IX(j, i) + 1] = (int16_t)-xi;
        }
    *xexp = s - F;
#undef IX
}

int or_inv_q15(int n, const int16_t* a, int16_t* x, int32_t* xexp, int32_t* sat_out)
{
    const size_t nn = (size_t)(n > 0 ? n : 1) * (size_t)(n > 0 ? n : 1);
    int64_t* rr = calloc(nn, sizeof(int64_t));
    int64_t* ri = calloc(nn, sizeof(int64_t));
    int64_t* yr = calloc(nn, sizeof(int64_t));
    int64_t* yi = calloc(nn, sizeof(int64_t));
    int32_t sat = 0;
    int info = 0;
#define IX(i, j) ((size_t)(i) * n + (j))

    /* eqs. (3)-(4), row by row */
    info = q15_factor(n, a, rr, ri, &sat);
    if (info) {
        memset(x, 0, sizeof(int16_t) * 2 * (size_t)n * n);
        *xexp = 0;
        *sat_out = sat;
        free(rr); free(ri); free(yr); free(yi);
        return info;
    }

    /* the exponent of Y = X 2^F */
    const int F = 2 * q15_log2_rmin(n, rr) - q15_ceil_log2(n);

    /* Section IV.A: R X = S with S's known upper triangle diag(1/r_ii); row i
     * from the bottom, its diagonal last (it needs x_ik, k > i, of its own
     * row through the mirror); s_i 2^(F+15) = 2^(F+30) / r_ii */
    for (int i = n - 1; i >= 0; --i) {
        const int64_t d = rr[IX(i, i)];
        const int64_t t = q_rdiv((int64_t)1 << (F + 30), d);
        for (int j = n - 1; j >= i; --j) {
            int64_t sr = (j == i) ? t : 0, si = 0;
            for (int k = i + 1; k < n; ++k) {
                int64_t xr, xi;                                /* x-hat_kj */
                if (k <= j) { xr = yr[IX(k, j)]; xi = yi[IX(k, j)]; }
                else        { xr = yr[IX(j, k)]; xi = -yi[IX(j, k)]; }
                sr -= rr[IX(i, k)] * xr - ri[IX(i, k)] * xi;
                si -= rr[IX(i, k)] * xi + ri[IX(i, k)] * xr;
            }
            yr[IX(i, j)] = q_clip(q_rdiv(sr, d), Y_LIM, &sat);
            yi[IX(i, j)] = (j == i) ? 0 : q_clip(q_rdiv(si, d), Y_LIM, &sat);
        }
    }

    /* int16 mantissas with one exponent: the smallest shift that fits */
    q15_emit(n, yr, yi, F, x, xexp);
    *sat_out = sat;
    free(rr); free(ri); free(yr); free(yi);
    return 0;
#undef IX
}

/* The Section III methods in the format above (variant 0: III.A, 1: III.B),
 * Cholesky only; arguments and results as or_inv_q15. */
int or_inv_q15_cmp(int variant, int n, const int16_t* a, int16_t* x, int32_t* xexp,
                   int32_t* sat_out)
{
    const size_t nn = (size_t)(n > 0 ? n : 1) * (size_t)(n > 0 ? n : 1);
    int64_t* rr = calloc(nn, sizeof(int64_t));
    int64_t* ri = calloc(nn, sizeof(int64_t));
    int64_t* yr = calloc(nn, sizeof(int64_t));
    int64_t* yi = calloc(nn, sizeof(int64_t));
    int64_t* wr = calloc(nn, sizeof(int64_t));
    int64_t* wi = calloc(nn, sizeof(int64_t));
    int32_t sat = 0;
#define IX(i, j) ((size_t)(i) * n + (j))
    const int info = q15_factor(n, a, rr, ri, &sat);
    if (info) {
        memset(x, 0, sizeof(int16_t) * 2 * (size_t)n * n);
        *xexp = 0;
        *sat_out = sat;
        free(rr); free(ri); free(yr); free(yi); free(wr); free(wi);
        return info;
    }
    const int b = q15_log2_rmin(n, rr), lg = q15_ceil_log2(n);
    const int F = 2 * b - lg;
    const int G = b + 13 - (lg + 1) / 2;

    if (variant == 0) {
        /* III.A: columns i = n-1..0; w holds the forward solution b 2^G */
        const int64_t up = (int64_t)1 << (F + 15 - G);
        for (int i = n - 1; i >= 0; --i) {
            for (int j = i; j < n; ++j) {
                int64_t sr = (j == i) ? ((int64_t)1 << (G + 15)) : 0, si = 0;
                for (int k = i; k < j; ++k) {                  /* conj(r_kj) b_k */
                    sr -= rr[IX(k, j)] * wr[k] + ri[IX(k, j)] * wi[k];
                    si -= rr[IX(k, j)] * wi[k] - ri[IX(k, j)] * wr[k];
                }
                wr[j] = q_clip(q_rdiv(sr, rr[IX(j, j)]), W_LIM, &sat);
                wi[j] = q_clip(q_rdiv(si, rr[IX(j, j)]), W_LIM, &sat);
            }
            for (int j = i; j >= 0; --j) {
                int64_t sr = (j == i) ? wr[j] * up : 0, si = (j == i) ? wi[j] * up : 0;
                for (int k = j + 1; k < n; ++k) {
                    int64_t hr, hi;                            /* x-hat_ki */
                    if (k <= i) { hr = yr[IX(k, i)]; hi = yi[IX(k, i)]; }
                    else        { hr = yr[IX(i, k)]; hi = -yi[IX(i, k)]; }
                    sr -= rr[IX(j, k)] * hr - ri[IX(j, k)] * hi;
                    si -= rr[IX(j, k)] * hi + ri[IX(j, k)] * hr;
                }
                yr[IX(j, i)] = q_clip(q_rdiv(sr, rr[IX(j, j)]), Y_LIM, &sat);
                yi[IX(j, i)] = (j == i) ? 0 : q_clip(q_rdiv(si, rr[IX(j, j)]), Y_LIM, &sat);
            }
        }
    } else {
        /* III.B: M = R^{-1} 2^G column by column (rows j = i..0) */
        for (int i = 0; i < n; ++i) {
            wr[IX(i, i)] = q_clip(q_rdiv((int64_t)1 << (G + 15), rr[IX(i, i)]), W_LIM, &sat);
            wi[IX(i, i)] = 0;
            for (int j = i - 1; j >= 0; --j) {
                int64_t sr = 0, si = 0;
                for (int k = j + 1; k <= i; ++k) {             /* r_jk m_ki */
                    sr -= rr[IX(j, k)] * wr[IX(k, i)] - ri[IX(j, k)] * wi[IX(k, i)];
                    si -= rr[IX(j, k)] * wi[IX(k, i)] + ri[IX(j, k)] * wr[IX(k, i)];
                }
                wr[IX(j, i)] = q_clip(q_rdiv(sr, rr[IX(j, j)]), W_LIM, &sat);
                wi[IX(j, i)] = q_clip(q_rdiv(si, rr[IX(j, j)]), W_LIM, &sat);
            }
        }
        /* X = M M^* upper half: x_ij = sum_{k >= j} m_ik conj(m_jk), i <= j */
        const int64_t down = (int64_t)1 << (2 * G - F);
        for (int i = 0; i < n; ++i)
            for (int j = i; j < n; ++j) {
                int64_t sr = 0, si = 0;
                for (int k = j; k < n; ++k) {
                    sr += wr[IX(i, k)] * wr[IX(j, k)] + wi[IX(i, k)] * wi[IX(j, k)];
                    si += wi[IX(i, k)] * wr[IX(j, k)] - wr[IX(i, k)] * wi[IX(j, k)];
                }
                yr[IX(i, j)] = q_clip(q_rdiv(sr, down), Y_LIM, &sat);
                yi[IX(i, j)] = (j == i) ? 0 : q_clip(q_rdiv(si, down), Y_LIM, &sat);
            }
    }
    q15_emit(n, yr, yi, F, x, xexp);
    *sat_out = sat;
    free(rr); free(ri); free(yr); free(yi); free(wr); free(wi);
    return 0;
#undef IX
}

void or_inv_q15_cmp_batched(int variant, long batch, int n, const int16_t* a, int16_t* x,
                            int32_t* xexp, int32_t* sat, int32_t* info)
{
    const size_t step = 2 * (size_t)n * n;
    for (long b = 0; b < batch; ++b)
        info[b] = or_inv_q15_cmp(variant, n, a + b * step, x + b * step, xexp + b, sat + b);
}

void or_inv_q15_batched(long batch, int n, const int16_t* a, int16_t* x, int32_t* xexp,
                        int32_t* sat, int32_t* info)
{
    const size_t step = 2 * (size_t)n * n;
    for (long b = 0; b < batch; ++b)
        info[b] = or_inv_q15(n, a + b * step, x + b * step, xexp + b, sat + b);
}
