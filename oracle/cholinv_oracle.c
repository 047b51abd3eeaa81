/*
 * cholinv_oracle.c -- plain, single-threaded FP64 CPU oracle for the matrix
 * inversion of Krishnamoorthy & Menon, "Matrix Inversion Using Cholesky
 * Decomposition" (arXiv:1111.4144).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark load this library.  It shares no code, header
 * or constant with the GPU library, and it is deliberately slow and obvious:
 * no blocking, no reordering beyond what the equations state, no BLAS.
 *
 * Build: gcc -O2 -std=c11 -ffp-contract=off -fno-fast-math -shared -fPIC
 *        (see build.py next to this file).
 *
 * Exported routines (suffix _d: real symmetric, _z: complex Hermitian):
 *   or_chol_*          Section II eqs. (3)-(4)
 *   or_ldl_*           Section II.A eqs. (10)-(11)
 *   or_chol_solve_*    Section II eqs. (5)-(7)
 *   or_ldl_solve_*     Section II.A eqs. (12)-(14)
 *   or_inv_prop_*      Section IV.A / IV.B, the proposed inversion
 *   or_inv_eqsolve_*   Section III.A, equation solving
 *   or_inv_tri_*       Section III.B, triangular matrix operations
 *   or_inv_nonherm_z   Section III.C, D^{-1} = D^* (D D^*)^{-1}
 *   or_grad_*          gA = -X Gh X (gradient of Re<G, A^{-1}>)
 *   or_ns_step_*       one Newton-Schulz step X + X(I - AX)
 *   or_gauss_jordan_*  brute-force inverse (independent route)
 *   or_herm_eig_z      cyclic Jacobi eigenvalues (for the 2-norm condition)
 *   or_count_reset / or_count_get   multiply counter (Table 1 convention)
 * Batched forms loop the single-matrix routine over a stack of matrices;
 * or_inv_prop_batched_omp_* runs the same loop with OpenMP over matrices
 * (each matrix still by the single-threaded routine), for the all-cores CPU
 * baseline, with or_set_threads choosing the thread count.
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

/* one counter per thread, so that the all-cores batch loop below races on
 * nothing; the counting tests read it from the thread that ran the routine */
static _Thread_local unsigned long long g_mults = 0;

void or_count_reset(void) { g_mults = 0; }
unsigned long long or_count_get(void) { return g_mults; }

/* ---- real instantiation ------------------------------------------------ */
#define T double
#define SFX(name) name##_d
#define CONJ(x) (x)
#define RE(x) (x)
#define NANT ((double)NAN)
#define ABS(x) fabs(x)
#include "cholinv_oracle_impl.h"
#undef T
#undef SFX
#undef CONJ
#undef RE
#undef NANT
#undef ABS

/* ---- complex instantiation --------------------------------------------- */
#define T double complex
#define SFX(name) name##_z
#define CONJ(x) conj(x)
#define RE(x) creal(x)
#define NANT CMPLX(NAN, NAN)
#define ABS(x) cabs(x)
#include "cholinv_oracle_impl.h"
#undef T
#undef SFX
#undef CONJ
#undef RE
#undef NANT
#undef ABS

/* ---- exported wrappers -------------------------------------------------- */
#define EXPORT_BOTH(SUF, T)                                                    \
int or_chol_##SUF(int n, const T* a, long lda, T* r, long ldr)                 \
{ return chol_##SUF(n, a, lda, r, ldr); }                                      \
int or_ldl_##SUF(int n, const T* a, long lda, T* r, long ldr, double* d,       \
                 int require_pos)                                              \
{ return ldl_##SUF(n, a, lda, r, ldr, d, require_pos); }                       \
void or_chol_solve_##SUF(int n, const T* r, long ldr, const T* y, T* x)        \
{ chol_solve_##SUF(n, r, ldr, y, x); }                                         \
void or_ldl_solve_##SUF(int n, const T* r, long ldr, const double* d,          \
                        const T* y, T* x)                                      \
{ ldl_solve_##SUF(n, r, ldr, d, y, x); }                                       \
int or_inv_prop_##SUF(int method, int n, const T* a, long lda, T* x, long ldx, \
                      int fill_lower)                                          \
{ return inv_prop_##SUF(method, n, a, lda, x, ldx, fill_lower); }              \
int or_inv_eqsolve_##SUF(int method, int n, const T* a, long lda, T* x,        \
                         long ldx)                                             \
{ return inv_eqsolve_##SUF(method, n, a, lda, x, ldx); }                       \
int or_inv_tri_##SUF(int n, const T* a, long lda, T* x, long ldx)              \
{ return inv_tri_##SUF(n, a, lda, x, ldx); }                                   \
void or_grad_##SUF(int n, const T* x, const T* g, T* ga)                       \
{ grad_##SUF(n, x, g, ga); }                                                   \
void or_ns_step_##SUF(int n, const T* a, long lda, const T* x, T* x1)          \
{ ns_step_##SUF(n, a, lda, x, x1); }                                           \
int or_gauss_jordan_##SUF(int n, const T* a, long lda, T* x, long ldx)         \
{ return gauss_jordan_##SUF(n, a, lda, x, ldx); }                              \
/* Batched proposed inversion: a stack of dense n x n matrices, stride n*n.  */ \
void or_inv_prop_batched_##SUF(int method, long batch, int n, const T* a,      \
                               T* x, int* info)                                \
{                                                                              \
    for (long b = 0; b < batch; ++b)                                           \
        info[b] = inv_prop_##SUF(method, n, a + b * (long)n * n, n,            \
                                 x + b * (long)n * n, n, 1);                   \
}                                                                              \
/* Packed variable-size batch: matrix b has order ns[b] and starts at        */ \
/* element offs[b]; it is dense with leading dimension ns[b].                 */ \
void or_inv_prop_varlen_##SUF(int method, long batch, const int* ns,           \
                              const long* offs, const T* a, T* x, int* info)   \
{                                                                              \
    for (long b = 0; b < batch; ++b)                                           \
        info[b] = inv_prop_##SUF(method, ns[b], a + offs[b], ns[b],            \
                                 x + offs[b], ns[b], 1);                       \
}                                                                              \
void or_inv_prop_batched_omp_##SUF(int method, long batch, int n, const T* a,  \
                                   T* x, int* info)                            \
{                                                                              \
    _Pragma("omp parallel for schedule(static)")                               \
    for (long b = 0; b < batch; ++b)                                           \
        info[b] = inv_prop_##SUF(method, n, a + b * (long)n * n, n,            \
                                 x + b * (long)n * n, n, 1);                   \
}                                                                              \
void or_grad_batched_##SUF(long batch, int n, const T* x, const T* g, T* ga)   \
{                                                                              \
    for (long b = 0; b < batch; ++b)                                           \
        grad_##SUF(n, x + b * (long)n * n, g + b * (long)n * n,                \
                   ga + b * (long)n * n);                                      \
}

EXPORT_BOTH(d, double)
EXPORT_BOTH(z, double complex)

#ifdef _OPENMP
#include <omp.h>
void or_set_threads(int t) { omp_set_num_threads(t > 0 ? t : 1); }
int or_max_threads(void) { return omp_get_max_threads(); }
#else
void or_set_threads(int t) { (void)t; }
int or_max_threads(void) { return 1; }
#endif

/* Section III.C: for an arbitrary square D, A = D D^* is Hermitian           */
/* positive definite when D is non-singular; D^{-1} = D^* A^{-1}.             */
int or_inv_nonherm_z(int n, const double complex* dm, double complex* dinv)
{
    size_t nn = (size_t)(n > 0 ? n * n : 1);
    double complex* a = (double complex*)malloc(sizeof(double complex) * nn);
    double complex* x = (double complex*)malloc(sizeof(double complex) * nn);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            double complex acc = 0;
            for (int k = 0; k < n; ++k) acc += dm[(long)i * n + k] * conj(dm[(long)j * n + k]);
            a[(long)i * n + j] = acc;
        }
    int info = inv_prop_z(0, n, a, n, x, n, 1);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            double complex acc = 0;
            for (int k = 0; k < n; ++k) acc += conj(dm[(long)k * n + i]) * x[(long)k * n + j];
            dinv[(long)i * n + j] = acc;
        }
    free(x);
    free(a);
    return info;
}

/*
 * Eigenvalues of a Hermitian matrix (upper triangle read) by the cyclic
 * Jacobi method on its real symmetric embedding [[Re A, -Im A], [Im A, Re A]],
 * whose spectrum is that of A with every eigenvalue repeated twice.  The
 * n eigenvalues are written to w in increasing order.  Used for the 2-norm
 * condition number kappa = w[n-1] / w[0] of a positive-definite input.
 */
int or_herm_eig_z(int n, const double complex* a, long lda, double* w)
{
    int m = 2 * n;
    double* s = (double*)malloc(sizeof(double) * (size_t)(m > 0 ? m * m : 1));
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            double complex v = herm_at_z(a, lda, i, j);
            s[(long)i * m + j] = creal(v);
            s[(long)(i + n) * m + (j + n)] = creal(v);
            s[(long)i * m + (j + n)] = -cimag(v);
            s[(long)(i + n) * m + j] = cimag(v);
        }
    int sweeps = 0;
    for (; sweeps < 100; ++sweeps) {
        double off = 0, tot = 0;
        for (int i = 0; i < m; ++i)
            for (int j = 0; j < m; ++j) {
                double v = s[(long)i * m + j] * s[(long)i * m + j];
                tot += v;
                if (i != j) off += v;
            }
        if (off <= 1e-30 * tot) break;
        for (int p = 0; p < m - 1; ++p)
            for (int q = p + 1; q < m; ++q) {
                double apq = s[(long)p * m + q];
                if (apq == 0.0) continue;
                double app = s[(long)p * m + p], aqq = s[(long)q * m + q];
                /* rotation angle that annihilates s_pq (Golub & Van Loan, Alg. 8.4.1) */
                double tau = (aqq - app) / (2.0 * apq);
                double t = (tau >= 0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                double c = 1.0 / sqrt(1.0 + t * t), sn = t * c;
                for (int k = 0; k < m; ++k) {          /* columns p, q */
                    double skp = s[(long)k * m + p], skq = s[(long)k * m + q];
                    s[(long)k * m + p] = c * skp - sn * skq;
                    s[(long)k * m + q] = sn * skp + c * skq;
                }
                for (int k = 0; k < m; ++k) {          /* rows p, q */
                    double spk = s[(long)p * m + k], sqk = s[(long)q * m + k];
                    s[(long)p * m + k] = c * spk - sn * sqk;
                    s[(long)q * m + k] = sn * spk + c * sqk;
                }
            }
    }
    double* ev = (double*)malloc(sizeof(double) * (size_t)(m > 0 ? m : 1));
    for (int i = 0; i < m; ++i) ev[i] = s[(long)i * m + i];
    for (int i = 1; i < m; ++i) {                      /* insertion sort */
        double v = ev[i];
        int j = i - 1;
        while (j >= 0 && ev[j] > v) { ev[j + 1] = ev[j]; --j; }
        ev[j + 1] = v;
    }
    for (int i = 0; i < n; ++i) w[i] = 0.5 * (ev[2 * i] + ev[2 * i + 1]);
    free(ev);
    free(s);
    return sweeps >= 100;
}
