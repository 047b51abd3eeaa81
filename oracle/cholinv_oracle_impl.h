/*
 * Type-generic body of the FP64 CPU oracle.  TEST INFRASTRUCTURE ONLY: it is
 * used by the tests, the smoke check and the CPU baseline of the benchmark,
 * never by the GPU library.
 *
 * This file is included twice by cholinv_oracle.c: once with T = double
 * (real symmetric input, suffix _d) and once with T = double complex
 * (Hermitian input, suffix _z).  The including file defines
 *   T          element type
 *   SFX(name)  name with the type suffix appended
 *   CONJ(x)    complex conjugate (identity for real)
 *   RE(x)      real part (identity for real)
 *   NANT       a NaN of type T (both parts NaN for complex)
 *   ABS(x)     absolute value
 *
 * Matrices are row major with a leading dimension (elements between rows).
 * Only the upper triangle (i <= j) of an input A is ever read; the imaginary
 * part of a diagonal entry is ignored.  Every sum runs over increasing k, as
 * the equations are written.  Indices are 0-based here; the paper's are
 * 1-based.
 *
 * Operation counter: every multiply that sits inside a sum of the paper's
 * equations increments the global counter g_mults (one per complex or real
 * multiply, the convention of the paper's operation counts).  Scalings,
 * divisions, square roots and the LDL helper products t_k are not counted.
 */

/* Hermitian entry a_kj of A rebuilt from the upper triangle. */
static T SFX(herm_at)(const T* a, long lda, int k, int j)
{
    if (k < j) return a[(long)k * lda + j];
    if (k > j) return CONJ(a[(long)j * lda + k]);
    return (T)RE(a[(long)k * lda + k]);
}

/* ------------------------------------------------------------------------ */
/* Section II, eqs. (3)-(4): Cholesky A = R^* R, R upper triangular.          */
/* Row i of R is computed from rows 0..i-1: first the diagonal pivot (eq. 3), */
/* then the entries right of it (eq. 4).  R's strict lower part is zeroed.    */
/* Returns 0, or i+1 for the first row whose radicand is not > 0 / finite.    */
/* ------------------------------------------------------------------------ */
static int SFX(chol)(int n, const T* a, long lda, T* r, long ldr)
{
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < i; ++j) r[(long)i * ldr + j] = 0;
    for (int i = 0; i < n; ++i) {
        /* eq. (3): r_ii = sqrt(a_ii - sum_{k<i} r_ki^* r_ki) */
        double rad = RE(a[(long)i * lda + i]);
        for (int k = 0; k < i; ++k) {
            T rki = r[(long)k * ldr + i];
            rad -= RE(CONJ(rki) * rki);
            g_mults++;
        }
        if (!(rad > 0.0) || !isfinite(rad)) return i + 1;
        double rii = sqrt(rad);
        r[(long)i * ldr + i] = rii;
        /* eq. (4): r_ij = (1/r_ii)(a_ij - sum_{k<i} r_ki^* r_kj), j > i */
        for (int j = i + 1; j < n; ++j) {
            T acc = a[(long)i * lda + j];
            for (int k = 0; k < i; ++k) {
                acc -= CONJ(r[(long)k * ldr + i]) * r[(long)k * ldr + j];
                g_mults++;
            }
            r[(long)i * ldr + j] = acc / rii;
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Section II.A, eqs. (10)-(11): LDL A = R^* D R, R unit upper triangular.    */
/* The efficient form: per row i the helper t_k = r_ki^* d_k is formed once,  */
/* so every term of the sums costs one multiply.                               */
/* require_pos = 1: a pivot d_i that is not > 0 (or not finite) fails, as the */
/* inversion of a positive-definite matrix needs; require_pos = 0: only a     */
/* zero or non-finite pivot fails.  Returns 0 or the 1-based failing row.     */
/* ------------------------------------------------------------------------ */
static int SFX(ldl)(int n, const T* a, long lda, T* r, long ldr, double* d,
                    int require_pos)
{
    T* t = (T*)malloc(sizeof(T) * (size_t)(n > 0 ? n : 1));
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < i; ++j) r[(long)i * ldr + j] = 0;
    int info = 0;
    for (int i = 0; i < n && !info; ++i) {
        for (int k = 0; k < i; ++k) t[k] = CONJ(r[(long)k * ldr + i]) * d[k];
        /* eq. (10): d_i = a_ii - sum_{k<i} r_ki^* r_ki d_k */
        double di = RE(a[(long)i * lda + i]);
        for (int k = 0; k < i; ++k) {
            di -= RE(t[k] * r[(long)k * ldr + i]);
            g_mults++;
        }
        int bad = require_pos ? !(di > 0.0) : (di == 0.0);
        if (bad || !isfinite(di)) { info = i + 1; break; }
        d[i] = di;
        r[(long)i * ldr + i] = 1;
        /* eq. (11): r_ij = (1/d_i)(a_ij - sum_{k<i} r_ki^* r_kj d_k), j > i */
        for (int j = i + 1; j < n; ++j) {
            T acc = a[(long)i * lda + j];
            for (int k = 0; k < i; ++k) {
                acc -= t[k] * r[(long)k * ldr + j];
                g_mults++;
            }
            r[(long)i * ldr + j] = acc / di;
        }
    }
    free(t);
    return info;
}

/* ------------------------------------------------------------------------ */
/* Section II, eqs. (5)-(7): solve A x = y with A = R^* R.                    */
/* R^* b = y is a forward substitution (R^* is lower), R x = b a backward one. */
/* ------------------------------------------------------------------------ */
static void SFX(chol_solve)(int n, const T* r, long ldr, const T* y, T* x)
{
    T* b = (T*)malloc(sizeof(T) * (size_t)(n > 0 ? n : 1));
    for (int i = 0; i < n; ++i) {                       /* eq. (6) */
        T acc = y[i];
        for (int k = 0; k < i; ++k) {
            acc -= CONJ(r[(long)k * ldr + i]) * b[k];
            g_mults++;
        }
        b[i] = acc / RE(r[(long)i * ldr + i]);
    }
    for (int i = n - 1; i >= 0; --i) {                  /* eq. (7) */
        T acc = b[i];
        for (int k = i + 1; k < n; ++k) {
            acc -= r[(long)i * ldr + k] * x[k];
            g_mults++;
        }
        x[i] = acc / RE(r[(long)i * ldr + i]);
    }
    free(b);
}

/* Section II.A, eqs. (12)-(14): A = R^* D R.  R^* D b = y is solved as        */
/* R^* c = y (unit lower) and b = D^{-1} c; then R x = b (unit upper).         */
static void SFX(ldl_solve)(int n, const T* r, long ldr, const double* d,
                           const T* y, T* x)
{
    T* c = (T*)malloc(sizeof(T) * (size_t)(n > 0 ? n : 1));
    for (int i = 0; i < n; ++i) {                       /* eq. (13) */
        T acc = y[i];
        for (int k = 0; k < i; ++k) {
            acc -= CONJ(r[(long)k * ldr + i]) * c[k];
            g_mults++;
        }
        c[i] = acc;
    }
    for (int i = n - 1; i >= 0; --i) {                  /* eq. (14) */
        T acc = c[i] / d[i];                            /* b_i */
        for (int k = i + 1; k < n; ++k) {
            acc -= r[(long)i * ldr + k] * x[k];
            g_mults++;
        }
        x[i] = acc;
    }
    free(c);
}

static void SFX(fill_nan)(int n, T* x, long ldx)
{
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) x[(long)i * ldx + j] = NANT;
}

static void SFX(mirror)(int n, T* x, long ldx)
{
    /* x_ji = x_ij^* for i < j (the Hermitian half "where needed") */
    for (int i = 0; i < n; ++i)
        for (int j = i + 1; j < n; ++j)
            x[(long)j * ldx + i] = CONJ(x[(long)i * ldx + j]);
}

/* Factor with the chosen method: method 0 = Cholesky, 1 = LDL (unit R and d). */
static int SFX(factor)(int method, int n, const T* a, long lda, T* r, double* d)
{
    if (method == 0) {
        int info = SFX(chol)(n, a, lda, r, n);
        if (!info)
            for (int i = 0; i < n; ++i) d[i] = RE(r[(long)i * n + i]);
        return info;
    }
    return SFX(ldl)(n, a, lda, r, n, d, 1);
}

/* ------------------------------------------------------------------------ */
/* Section IV: the proposed inversion.                                        */
/* Cholesky (IV.A): R X = B with B = R^{*-1} lower triangular; its upper       */
/* triangle including the diagonal is S = diag(1/r_ii) (eq. 24), so the first */
/* triangular solve is skipped and the upper half of X follows from           */
/*   x_ij = (delta_ij s_ii - sum_{k>i} r_ik xh_kj) / r_ii,  i <= j,            */
/* where xh_kj = x_kj for k <= j and x_jk^* for k > j (already computed).      */
/* LDL (IV.B): R unit, S~ = diag(1/d_i) (eq. 29), no division:                 */
/*   x_ij = delta_ij / d_i - sum_{k>i} r_ik xh_kj.                            */
/* Columns j = n-1..0, rows i = j..0.  x_ii is real.  fill_lower mirrors.      */
/* On failure X is filled with NaN and the 1-based failing pivot returned.    */
/* ------------------------------------------------------------------------ */
static int SFX(inv_prop)(int method, int n, const T* a, long lda, T* x, long ldx,
                         int fill_lower)
{
    T* r = (T*)malloc(sizeof(T) * (size_t)(n > 0 ? n * n : 1));
    double* d = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    int info = SFX(factor)(method, n, a, lda, r, d);
    if (info) {
        SFX(fill_nan)(n, x, ldx);
    } else {
        for (int j = n - 1; j >= 0; --j) {
            for (int i = j; i >= 0; --i) {
                /* s_ii = 1/r_ii (eq. 24) or 1/d_i (eq. 29) */
                T acc = (i == j) ? (T)(1.0 / d[i]) : (T)0;
                for (int k = i + 1; k < n; ++k) {
                    T xh = (k <= j) ? x[(long)k * ldx + j] : CONJ(x[(long)j * ldx + k]);
                    acc -= r[(long)i * n + k] * xh;
                    g_mults++;
                }
                T v = (method == 0) ? acc / d[i] : acc;
                if (i == j) v = RE(v);
                x[(long)i * ldx + j] = v;
            }
        }
        if (fill_lower) SFX(mirror)(n, x, ldx);
    }
    free(r);
    free(d);
    return info;
}

/* ------------------------------------------------------------------------ */
/* Section III.A: equation solving, A x_i = e_i (eq. 15), upper half only.    */
/* For column i: forward R^* b = e_i for rows j >= i (the sums run over every */
/* k < j; the zero entries b_k, k < i, are not skipped), then backward        */
/* R x = b for rows j = i..0, taking xh_ki = x_ik^* for k > i from columns    */
/* already solved (columns run i = n-1..0).  LDL: R^* c = e_i, b = D^{-1} c.   */
/* ------------------------------------------------------------------------ */
static int SFX(inv_eqsolve)(int method, int n, const T* a, long lda, T* x, long ldx)
{
    T* r = (T*)malloc(sizeof(T) * (size_t)(n > 0 ? n * n : 1));
    double* d = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    T* f = (T*)malloc(sizeof(T) * (size_t)(n > 0 ? n : 1));
    int info = SFX(factor)(method, n, a, lda, r, d);
    if (info) {
        SFX(fill_nan)(n, x, ldx);
    } else {
        for (int i = n - 1; i >= 0; --i) {
            /* f: the forward unknowns; Cholesky: b itself, LDL: c = D b. */
            for (int j = 0; j < i; ++j) f[j] = 0;
            for (int j = i; j < n; ++j) {
                T acc = (j == i) ? (T)1 : (T)0;
                for (int k = 0; k < j; ++k) {
                    acc -= CONJ(r[(long)k * n + j]) * f[k];
                    g_mults++;
                }
                f[j] = (method == 0) ? acc / d[j] : acc;   /* l_jj = r_jj, or unit */
            }
            for (int j = i; j >= 0; --j) {
                T acc = (method == 0) ? f[j] : f[j] / d[j];   /* b_j */
                for (int k = j + 1; k < n; ++k) {
                    T xh = (k <= i) ? x[(long)k * ldx + i] : CONJ(x[(long)i * ldx + k]);
                    acc -= r[(long)j * n + k] * xh;
                    g_mults++;
                }
                T v = (method == 0) ? acc / d[j] : acc;
                if (j == i) v = RE(v);
                x[(long)j * ldx + i] = v;
            }
        }
        SFX(mirror)(n, x, ldx);
    }
    free(f);
    free(r);
    free(d);
    return info;
}

/* ------------------------------------------------------------------------ */
/* Section III.B: triangular operations, A^{-1} = R^{-1} R^{*-1} (eq. 17).    */
/* M = R^{-1} column by column from R m_i = e_i (eq. 18), rows j = i..0, sums  */
/* over every k > j (the zeros m_ki, k > i, are not skipped); then the upper  */
/* half of X = M M^* (eq. 19), whose sums skip M's zeros (k >= j).            */
/* ------------------------------------------------------------------------ */
static int SFX(inv_tri)(int n, const T* a, long lda, T* x, long ldx)
{
    T* r = (T*)malloc(sizeof(T) * (size_t)(n > 0 ? n * n : 1));
    T* m = (T*)calloc((size_t)(n > 0 ? n * n : 1), sizeof(T));
    int info = SFX(chol)(n, a, lda, r, n);
    if (info) {
        SFX(fill_nan)(n, x, ldx);
    } else {
        for (int i = 0; i < n; ++i) {
            for (int j = i; j >= 0; --j) {
                T acc = (j == i) ? (T)1 : (T)0;
                for (int k = j + 1; k < n; ++k) {
                    acc -= r[(long)j * n + k] * m[(long)k * n + i];
                    g_mults++;
                }
                m[(long)j * n + i] = acc / RE(r[(long)j * n + j]);
            }
        }
        for (int i = 0; i < n; ++i) {
            for (int j = i; j < n; ++j) {
                T acc = 0;
                for (int k = j; k < n; ++k) {
                    acc += m[(long)i * n + k] * CONJ(m[(long)j * n + k]);
                    g_mults++;
                }
                if (i == j) acc = RE(acc);
                x[(long)i * ldx + j] = acc;
            }
        }
        SFX(mirror)(n, x, ldx);
    }
    free(m);
    free(r);
    return info;
}

/* ------------------------------------------------------------------------ */
/* Gradient of the real loss L = Re <G, X>, X = A^{-1}, along Hermitian        */
/* perturbations of A: from d(A^{-1}) = -A^{-1} dA A^{-1},                     */
/*   gA = -X Gh X,  Gh = (G + G^H)/2   (X is Hermitian).                       */
/* Plain dense products; x is the full Hermitian inverse.                     */
/* ------------------------------------------------------------------------ */
static void SFX(grad)(int n, const T* x, const T* g, T* ga)
{
    T* gh = (T*)malloc(sizeof(T) * (size_t)(n > 0 ? n * n : 1));
    T* t = (T*)malloc(sizeof(T) * (size_t)(n > 0 ? n * n : 1));
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j)
            gh[(long)i * n + j] = 0.5 * (g[(long)i * n + j] + CONJ(g[(long)j * n + i]));
    for (int i = 0; i < n; ++i)                 /* t = Gh X */
        for (int j = 0; j < n; ++j) {
            T acc = 0;
            for (int k = 0; k < n; ++k) acc += gh[(long)i * n + k] * x[(long)k * n + j];
            t[(long)i * n + j] = acc;
        }
    for (int i = 0; i < n; ++i)                 /* ga = -X t */
        for (int j = 0; j < n; ++j) {
            T acc = 0;
            for (int k = 0; k < n; ++k) acc += x[(long)i * n + k] * t[(long)k * n + j];
            ga[(long)i * n + j] = -acc;
        }
    free(t);
    free(gh);
}

/* One Newton-Schulz step X1 = X + X (I - A X) (= X(2I - AX)), with the       */
/* Hermitian A rebuilt from its upper triangle.  Plain dense products.        */
static void SFX(ns_step)(int n, const T* a, long lda, const T* x, T* x1)
{
    T* e = (T*)malloc(sizeof(T) * (size_t)(n > 0 ? n * n : 1));
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            T acc = (i == j) ? (T)1 : (T)0;
            for (int k = 0; k < n; ++k) acc -= SFX(herm_at)(a, lda, i, k) * x[(long)k * n + j];
            e[(long)i * n + j] = acc;
        }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            T acc = x[(long)i * n + j];
            for (int k = 0; k < n; ++k) acc += x[(long)i * n + k] * e[(long)k * n + j];
            x1[(long)i * n + j] = acc;
        }
    free(e);
}

/* Brute force: Gauss-Jordan elimination with partial pivoting on [A | I].    */
/* Independent of every Cholesky route; for tiny n.  Returns 0 or 1 if        */
/* singular.                                                                  */
static int SFX(gauss_jordan)(int n, const T* a, long lda, T* x, long ldx)
{
    int w = 2 * n;
    T* m = (T*)malloc(sizeof(T) * (size_t)(n > 0 ? n * w : 1));
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < w; ++j)
            m[(long)i * w + j] = (j < n) ? SFX(herm_at)(a, lda, i, j) : (T)((j - n == i) ? 1 : 0);
    int info = 0;
    for (int c = 0; c < n; ++c) {
        int p = c;
        for (int i = c + 1; i < n; ++i)
            if (ABS(m[(long)i * w + c]) > ABS(m[(long)p * w + c])) p = i;
        if (m[(long)p * w + c] == 0) { info = 1; break; }
        if (p != c)
            for (int j = 0; j < w; ++j) {
                T t = m[(long)p * w + j];
                m[(long)p * w + j] = m[(long)c * w + j];
                m[(long)c * w + j] = t;
            }
        T piv = m[(long)c * w + c];
        for (int j = 0; j < w; ++j) m[(long)c * w + j] /= piv;
        for (int i = 0; i < n; ++i) {
            if (i == c) continue;
            T f = m[(long)i * w + c];
            for (int j = 0; j < w; ++j) m[(long)i * w + j] -= f * m[(long)c * w + j];
        }
    }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j)
            x[(long)i * ldx + j] = info ? NANT : m[(long)i * w + n + j];
    free(m);
    return info;
}
