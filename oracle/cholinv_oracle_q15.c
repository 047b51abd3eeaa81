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

int or_inv_q15(int n, const int16_t* a, int16_t* x, int32_t* xexp, int32_t* sat_out)
{
    const size_t nn = (size_t)(n > 0 ? n : 1) * (size_t)(n > 0 ? n : 1);
    int64_t* rr = calloc(nn, sizeof(int64_t));
    int64_t* ri = calloc(nn, sizeof(int64_t));
    int64_t* yr = calloc(nn, sizeof(int64_t));
    int64_t* yi = calloc(nn, sizeof(int64_t));
    int32_t sat = 0;
    int info = 0;
#define A_RE(i, j) ((int64_t)a[2 * ((size_t)(i) * n + (j))])
#define A_IM(i, j) ((int64_t)a[2 * ((size_t)(i) * n + (j)) + 1])
#define IX(i, j) ((size_t)(i) * n + (j))

    /* eqs. (3)-(4), row by row */
    for (int i = 0; i < n; ++i) {
        int64_t acc = A_RE(i, i) * 32768;                      /* Q30 */
        for (int k = 0; k < i; ++k)
            acc -= rr[IX(k, i)] * rr[IX(k, i)] + ri[IX(k, i)] * ri[IX(k, i)];
        if (acc <= 0) {
            info = i + 1;
            break;
        }
        const int64_t d = q_isqrt(acc);                        /* Q15, >= 1 */
        rr[IX(i, i)] = d;
        ri[IX(i, i)] = 0;
        for (int j = i + 1; j < n; ++j) {
            int64_t sr = A_RE(i, j) * 32768, si = A_IM(i, j) * 32768;
            for (int k = 0; k < i; ++k) {                      /* conj(r_ki) r_kj */
                sr -= rr[IX(k, i)] * rr[IX(k, j)] + ri[IX(k, i)] * ri[IX(k, j)];
                si -= rr[IX(k, i)] * ri[IX(k, j)] - ri[IX(k, i)] * rr[IX(k, j)];
            }
            rr[IX(i, j)] = q_clip(q_rdiv(sr, d), Q15_MAX, &sat);
            ri[IX(i, j)] = q_clip(q_rdiv(si, d), Q15_MAX, &sat);
        }
    }
    if (info) {
        memset(x, 0, sizeof(int16_t) * 2 * (size_t)n * n);
        *xexp = 0;
        *sat_out = sat;
        free(rr); free(ri); free(yr); free(yi);
        return info;
    }

    /* the exponent of Y = X 2^F */
    int64_t rmin = Q15_MAX;
    for (int i = 0; i < n; ++i)
        if (rr[IX(i, i)] < rmin) rmin = rr[IX(i, i)];
    int b = 0;
    while ((rmin >> (b + 1)) > 0) ++b;                         /* 2^b <= rmin */
    int lg = 0;
    while ((1 << lg) < n) ++lg;
    const int F = 2 * b - lg;

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
    *sat_out = sat;
    free(rr); free(ri); free(yr); free(yi);
    return 0;
#undef A_RE
#undef A_IM
#undef IX
}

void or_inv_q15_batched(long batch, int n, const int16_t* a, int16_t* x, int32_t* xexp,
                        int32_t* sat, int32_t* info)
{
    const size_t step = 2 * (size_t)n * n;
    for (long b = 0; b < batch; ++b)
        info[b] = or_inv_q15(n, a + b * step, x + b * step, xexp + b, sat + b);
}
