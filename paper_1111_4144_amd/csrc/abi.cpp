// abi.cpp -- the C-ABI of libcholinv (declared in include/cholinv.h):
// argument checks, dispatch to the kernel families, error mapping.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>

#include "ci_launch.hpp"
#include "ci_large.hpp"
#include "ci_nonherm.hpp"
#include "ci_q15.hpp"
#include "ci_compare.hpp"
#include "cholinv.h"

namespace {

int map_err(hipError_t e)
{
    if (e == hipSuccess) return 0;
    if (e == hipErrorNotSupported) return CI_ERR_UNSUPPORTED;
    return CI_ERR_LAUNCH - (int)e;
}

bool valid_dtype(int d) { return d >= CI_F32 && d <= CI_C128; }

bool is_f32(int d) { return d == CI_F32 || d == CI_C64; }

size_t elem_size(int d)
{
    switch (d) {
    case CI_F32: return 4;
    case CI_F64: return 8;
    case CI_C64: return 8;
    case CI_C128: return 16;
    default: return 0;
    }
}

ci_opts default_opts() { return ci_opts{CI_METHOD_CHOL, CI_PLAIN, 0, 1}; }

// Returns 0 or the negative index (relative to `base`) of the bad option.
int check_opts(const ci_opts& o, int dtype)
{
    if (o.method != CI_METHOD_CHOL && o.method != CI_METHOD_LDL) return 1;
    if (o.precision != CI_PLAIN && o.precision != CI_MIXED) return 1;
    if (o.precision == CI_MIXED && !is_f32(dtype)) return 1;
    if (o.ns_steps < 0 || o.ns_steps > 3) return 1;
    if (o.precision == CI_PLAIN && o.ns_steps != 0) return 1;
    if (o.fill_lower != 0 && o.fill_lower != 1) return 1;
    return 0;
}

hipError_t run_small_one(int dtype, int64_t n, int op, int method, int mixed,
                         const ci::BatchArgs& p, hipStream_t s)
{
    if (op == ci::OP_INV) {
        const int eng = ci::tuned_engine(dtype, mixed, method, (int)n);
        if (eng != ci::ENG_DEFAULT)
            return ci::launch_engine(eng, dtype, (int)n, op, method, mixed, p, s);
    }
    if (n <= ci::tpm_nmax(dtype, mixed)) return ci::launch_tpm(dtype, (int)n, op, method, mixed, p, s);
    return ci::launch_group(dtype, (int)n, op, method, mixed, p, s);
}

// A dispatch's grid counts work-items in 32 bits.  The batched kernels use at
// most 256 lanes per matrix, so batches are launched in pieces of at most
// 2^22 matrices (2^30 work-items).
constexpr int64_t SMALL_CHUNK = (int64_t)1 << 22;

hipError_t run_small(int dtype, int64_t n, int op, int method, int mixed, const ci::BatchArgs& p,
                     hipStream_t s)
{
    if (p.batch <= SMALL_CHUNK) return run_small_one(dtype, n, op, method, mixed, p, s);
    const size_t es = elem_size(dtype);
    const size_t rs = (dtype == CI_F32 || dtype == CI_C64) ? 4 : 8;   // LDL pivot type
    for (int64_t b0 = 0; b0 < p.batch; b0 += SMALL_CHUNK) {
        ci::BatchArgs q = p;
        q.batch = std::min(SMALL_CHUNK, p.batch - b0);
        q.a = static_cast<const char*>(p.a) + (size_t)(b0 * p.sa) * es;
        q.x = static_cast<char*>(p.x) + (size_t)(b0 * p.sx) * es;
        q.info = p.info ? p.info + b0 : nullptr;
        q.dout = p.dout ? static_cast<char*>(p.dout) + (size_t)(b0 * n) * rs : nullptr;
        const hipError_t e = run_small_one(dtype, n, op, method, mixed, q, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace

extern "C" {

int chol_factor(int dtype, int64_t batch, int64_t n, void* a, int64_t lda, int64_t stride,
                int32_t* info, void* work, size_t work_bytes, void* stream)
{
    if (!valid_dtype(dtype)) return -1;
    if (batch < 0) return -2;
    if (n < 0 || (batch > 1 && n > CI_SMALL_NMAX)) return -3;
    if (batch > 0 && n > 0 && !a) return -4;
    if (lda < std::max<int64_t>(1, n)) return -5;
    if (batch > 1 && stride < lda * n) return -6;
    hipStream_t s = (hipStream_t)stream;
    if (batch == 0) return 0;
    if (n == 0) return info ? map_err(ci::fill_i32(info, batch, 0, s)) : 0;
    if (n > CI_SMALL_NMAX) {
        size_t need = ci::large_workspace(dtype, n, ci::LG_FACTOR, 0);
        if (work_bytes < need || (need && !work)) return CI_ERR_WORKSPACE;
        return map_err(ci::large_factor(dtype, n, a, lda, info, work, s,
                                        ci::tuned_large(dtype, 0, CI_METHOD_CHOL, n)));
    }
    ci::BatchArgs p{a, a, batch, lda, batch > 1 ? stride : lda * n, lda,
                    batch > 1 ? stride : lda * n, 0, 0, info, nullptr};
    return map_err(run_small(dtype, n, ci::OP_CHOL_FACTOR, 0, 0, p, s));
}

int ldl_factor(int dtype, int64_t batch, int64_t n, void* a, int64_t lda, int64_t stride,
               void* d, int32_t* info, void* stream)
{
    if (!valid_dtype(dtype)) return -1;
    if (batch < 0) return -2;
    if (n < 0 || n > CI_SMALL_NMAX) return -3;
    if (batch > 0 && n > 0 && !a) return -4;
    if (lda < std::max<int64_t>(1, n)) return -5;
    if (batch > 1 && stride < lda * n) return -6;
    if (batch > 0 && n > 0 && !d) return -7;
    hipStream_t s = (hipStream_t)stream;
    if (batch == 0) return 0;
    if (n == 0) return info ? map_err(ci::fill_i32(info, batch, 0, s)) : 0;
    ci::BatchArgs p{a, a, batch, lda, batch > 1 ? stride : lda * n, lda,
                    batch > 1 ? stride : lda * n, 0, 0, info, d};
    return map_err(run_small(dtype, n, ci::OP_LDL_FACTOR, 1, 0, p, s));
}

int chol_solve(int dtype, int method, int64_t batch, int64_t n, int64_t nrhs, const void* r,
               int64_t ldr, int64_t stride_r, const void* d, const void* b, int64_t ldb,
               int64_t stride_b, void* x, int64_t ldx, int64_t stride_x, void* stream)
{
    if (!valid_dtype(dtype)) return -1;
    if (method != CI_METHOD_CHOL && method != CI_METHOD_LDL) return -2;
    if (batch < 0) return -3;
    if (n < 0 || n > CI_SMALL_NMAX) return -4;
    if (nrhs < 0 || nrhs > INT32_MAX) return -5;
    const bool work = batch > 0 && n > 0 && nrhs > 0;
    if (work && !r) return -6;
    if (ldr < std::max<int64_t>(1, n)) return -7;
    if (batch > 1 && stride_r < ldr * n) return -8;
    if (work && method == CI_METHOD_LDL && !d) return -9;
    if (work && !b) return -10;
    if (ldb < std::max<int64_t>(1, nrhs)) return -11;
    if (batch > 1 && stride_b < ldb * n) return -12;
    if (work && !x) return -13;
    if (ldx < std::max<int64_t>(1, nrhs)) return -14;
    if (batch > 1 && stride_x < ldx * n) return -15;
    if (x == b && (ldx != ldb || (batch > 1 && stride_x != stride_b))) return -13;
    if (!work) return 0;
    // one lane per right-hand side: pieces of at most 2^30 right-hand sides
    // per launch (the grid counts work-items in 32 bits)
    const int64_t chunk = std::max<int64_t>(1, ((int64_t)1 << 30) / nrhs);
    const size_t es = elem_size(dtype), rs = (dtype == CI_F32 || dtype == CI_C64) ? 4 : 8;
    for (int64_t b0 = 0; b0 < batch; b0 += chunk) {
        const int64_t cnt = std::min(chunk, batch - b0);
        const int64_t sr = batch > 1 ? stride_r : 0, sb = batch > 1 ? stride_b : 0,
                      sx = batch > 1 ? stride_x : 0;
        ci::SolveArgs p{static_cast<const char*>(r) + (size_t)(b0 * sr) * es, ldr, sr,
                        d ? static_cast<const char*>(d) + (size_t)(b0 * n) * rs : nullptr,
                        static_cast<const char*>(b) + (size_t)(b0 * sb) * es, ldb, sb,
                        static_cast<char*>(x) + (size_t)(b0 * sx) * es, ldx, sx, cnt, (int)n,
                        (int)nrhs};
        const int rc = map_err(ci::launch_solve(dtype, method, p, (hipStream_t)stream));
        if (rc) return rc;
    }
    return 0;
}

int chol_inverse_nonherm(int dtype, int64_t batch, int64_t n, const void* d, int64_t stride,
                         void* x, const ci_opts* opts, void* work, size_t work_bytes,
                         int32_t* info, void* stream)
{
    if (!valid_dtype(dtype)) return -1;
    if (batch < 0) return -2;
    if (n < 0 || n > CI_SMALL_NMAX) return -3;
    if (batch > 0 && n > 0 && !d) return -4;
    if (batch > 1 && stride < n * n) return -5;
    if (batch > 0 && n > 0 && (!x || x == d)) return -6;
    ci_opts o = opts ? *opts : default_opts();
    if (check_opts(o, dtype)) return -7;
    hipStream_t s = (hipStream_t)stream;
    if (batch == 0) return 0;
    if (n == 0) return info ? map_err(ci::fill_i32(info, batch, 0, s)) : 0;
    const size_t need = chol_workspace_size(CI_FN_NONHERM, dtype, batch, n, &o);
    if (work_bytes < need || !work) return CI_ERR_WORKSPACE;
    const int64_t nn = n * n;
    const int64_t sd = batch > 1 ? stride : nn;
    const size_t es = elem_size(dtype);
    // one lane per entry in the product kernels: pieces of 2^18 matrices
    // (at most 2^30 work-items at order 64)
    constexpr int64_t chunk = (int64_t)1 << 18;
    for (int64_t b0 = 0; b0 < batch; b0 += chunk) {
        const int64_t cnt = std::min(chunk, batch - b0);
        const void* dc = static_cast<const char*>(d) + (size_t)(b0 * sd) * es;
        void* xc = static_cast<char*>(x) + (size_t)(b0 * sd) * es;
        void* a = static_cast<char*>(work) + (size_t)(b0 * nn) * es;
        void* xa = static_cast<char*>(work) + need / 2 + (size_t)(b0 * nn) * es;
        hipError_t e = ci::launch_gram(dtype, dc, sd, a, cnt, (int)n, s);
        if (e != hipSuccess) return map_err(e);
        // X_A = (D D^*)^{-1}, written in full (both halves feed the product)
        ci::BatchArgs p{a, xa, cnt, n, nn, n, nn, o.ns_steps, 1, info ? info + b0 : nullptr,
                        nullptr};
        e = run_small(dtype, n, ci::OP_INV, o.method, o.precision == CI_MIXED, p, s);
        if (e != hipSuccess) return map_err(e);
        e = ci::launch_adjoint_product(dtype, dc, sd, xa, xc, sd, cnt, (int)n, s);
        if (e != hipSuccess) return map_err(e);
    }
    return 0;
}

// Q15 batches for either route; k shifts the argument numbers of the errors
// (the compare entry point takes the variant first).
static int q15_run(int variant, int k, int64_t batch, int64_t n, const int16_t* a, int64_t stride,
                   int16_t* x, int32_t* xexp, int32_t* sat, int32_t* info, void* stream)
{
    if (batch < 0) return -(1 + k);
    if (n < 0 || n > CI_Q15_NMAX) return -(2 + k);
    const bool work = batch > 0 && n > 0;
    if (work && !a) return -(3 + k);
    if (batch > 1 && stride < n * n) return -(4 + k);
    if (work && (!x || x == a)) return -(5 + k);
    if (work && !xexp) return -(6 + k);
    if (!work) return (batch > 0 && info) ? map_err(ci::fill_i32(info, batch, 0, (hipStream_t)stream)) : 0;
    // one lane per matrix: pieces of 2^30 matrices per launch
    const int64_t st = batch > 1 ? stride : n * n;
    constexpr int64_t chunk = (int64_t)1 << 30;
    for (int64_t b0 = 0; b0 < batch; b0 += chunk) {
        const int64_t cnt = std::min(chunk, batch - b0);
        const int rc = map_err(ci::launch_inv_q15(a + 2 * b0 * st, st, x + 2 * b0 * st, xexp + b0,
                                                  sat ? sat + b0 : nullptr,
                                                  info ? info + b0 : nullptr, cnt, (int)n,
                                                  (hipStream_t)stream, variant));
        if (rc) return rc;
    }
    return 0;
}

int chol_inverse_q15(int64_t batch, int64_t n, const int16_t* a, int64_t stride, int16_t* x,
                     int32_t* xexp, int32_t* sat, int32_t* info, void* stream)
{
    return q15_run(0, 0, batch, n, a, stride, x, xexp, sat, info, stream);
}

int chol_inverse_q15_compare(int variant, int64_t batch, int64_t n, const int16_t* a,
                             int64_t stride, int16_t* x, int32_t* xexp, int32_t* sat,
                             int32_t* info, void* stream)
{
    if (variant != CI_III_A && variant != CI_III_B) return -1;
    return q15_run(variant == CI_III_A ? 1 : 2, 1, batch, n, a, stride, x, xexp, sat, info,
                   stream);
}

int chol_inverse_compare(int dtype, int variant, int method, int64_t batch, int64_t n,
                         const void* a, int64_t stride, void* x, int32_t* info, void* stream)
{
    if (!valid_dtype(dtype)) return -1;
    if (variant != CI_III_A && variant != CI_III_B && variant != CI_IV_SAME) return -2;
    if (method != CI_METHOD_CHOL && (method != CI_METHOD_LDL || variant == CI_III_B)) return -3;
    if (batch < 0) return -4;
    if (n < 0 || n > CI_COMPARE_NMAX) return -5;
    const bool work = batch > 0 && n > 0;
    if (work && !a) return -6;
    if (batch > 1 && stride < n * n) return -7;
    if (work && (!x || x == a)) return -8;
    hipStream_t s = (hipStream_t)stream;
    if (!work) return (batch > 0 && info) ? map_err(ci::fill_i32(info, batch, 0, s)) : 0;
    const int ldl = method == CI_METHOD_LDL ? 1 : 0;
    const int k = variant == CI_III_B ? 2 : (variant == CI_IV_SAME ? 3 + ldl : ldl);
    const int64_t st = batch > 1 ? stride : n * n;
    const size_t es = elem_size(dtype);
    constexpr int64_t chunk = (int64_t)1 << 30;          // one lane per matrix
    for (int64_t b0 = 0; b0 < batch; b0 += chunk) {
        const int64_t cnt = std::min(chunk, batch - b0);
        const int rc = map_err(ci::launch_compare(
            dtype, k, static_cast<const char*>(a) + (size_t)(b0 * st) * es, st,
            static_cast<char*>(x) + (size_t)(b0 * st) * es, st, info ? info + b0 : nullptr, cnt,
            (int)n, s));
        if (rc) return rc;
    }
    return 0;
}

int chol_inverse(int dtype, int64_t n, const void* a, int64_t lda, void* x, int64_t ldx,
                 const ci_opts* opts, void* work, size_t work_bytes, int32_t* info, void* stream)
{
    if (!valid_dtype(dtype)) return -1;
    if (n < 0) return -2;
    if (n > 0 && !a) return -3;
    if (lda < std::max<int64_t>(1, n)) return -4;
    if (n > 0 && !x) return -5;
    if (ldx < std::max<int64_t>(1, n)) return -6;
    ci_opts o = opts ? *opts : default_opts();
    if (check_opts(o, dtype)) return -7;
    hipStream_t s = (hipStream_t)stream;
    if (n == 0) return info ? map_err(ci::fill_i32(info, 1, 0, s)) : 0;
    if (n > CI_SMALL_NMAX) {
        if (a == x) return -5;
        size_t need = ci::large_workspace(dtype, n, ci::LG_INVERSE, o.precision == CI_MIXED);
        if (work_bytes < need || (need && !work)) return CI_ERR_WORKSPACE;
        if (o.method != CI_METHOD_CHOL) return CI_ERR_UNSUPPORTED;
        return map_err(ci::large_inverse(
            dtype, n, a, lda, x, ldx, o.precision == CI_MIXED, o.ns_steps, o.fill_lower, info, work,
            s, ci::tuned_large(dtype, o.precision == CI_MIXED, o.method, n)));
    }
    if (a == x && (o.precision == CI_MIXED || lda != ldx)) return -5;
    ci::BatchArgs p{a, x, 1, lda, lda * n, ldx, ldx * n, o.ns_steps, o.fill_lower, info, nullptr};
    return map_err(run_small(dtype, n, ci::OP_INV, o.method, o.precision == CI_MIXED, p, s));
}

int chol_inverse_batched(int dtype, int64_t batch, int64_t n_uniform, const int32_t* n_dev,
                         const int64_t* offsets_dev, int64_t n_max, const void* a,
                         int64_t stride_a, void* x, int64_t stride_x, const ci_opts* opts,
                         void* work, size_t work_bytes, int32_t* info, void* stream)
{
    if (!valid_dtype(dtype)) return -1;
    if (batch < 0) return -2;
    if (n_uniform < 0 || n_uniform > CI_SMALL_NMAX) return -3;
    const bool varlen = n_uniform == 0;
    if (varlen && batch > 0 && !n_dev) return -4;
    if (varlen && batch > 0 && !offsets_dev) return -5;
    if (varlen && (n_max < 1 || n_max > CI_SMALL_NMAX)) return -6;
    if (batch > 0 && !a) return -7;
    if (!varlen && stride_a < n_uniform * n_uniform) return -8;
    if (batch > 0 && !x) return -9;
    if (!varlen && stride_x < n_uniform * n_uniform) return -10;
    ci_opts o = opts ? *opts : default_opts();
    if (check_opts(o, dtype)) return -11;
    hipStream_t s = (hipStream_t)stream;
    if (batch == 0) return 0;
    if (a == x && o.precision == CI_MIXED) return -9;
    if (varlen) {
        size_t need = ci::varlen_workspace(batch);
        if (work_bytes < need || !work) return CI_ERR_WORKSPACE;
        return map_err(ci::launch_varlen(
            dtype, batch, n_dev, offsets_dev, (int)n_max, a, x, o.method, o.precision == CI_MIXED,
            o.ns_steps, o.fill_lower, info, work, s,
            ci::tuned_varlen(dtype, o.precision == CI_MIXED, o.method)));
    }
    ci::BatchArgs p{a, x, batch, n_uniform, stride_a, n_uniform, stride_x, o.ns_steps,
                    o.fill_lower, info, nullptr};
    return map_err(run_small(dtype, n_uniform, ci::OP_INV, o.method, o.precision == CI_MIXED, p, s));
}

int chol_inverse_batched_noalloc(int dtype, int64_t batch, int64_t n_uniform,
                                 const int32_t* n_dev, const int64_t* offsets_dev, int64_t n_max,
                                 const void* a, int64_t stride_a, void* x, int64_t stride_x,
                                 const ci_opts* opts, int32_t* info, void* stream)
{
    if (n_uniform == 0 && batch > CI_NOALLOC_MAX_BATCH) return CI_ERR_NOALLOC_LIMIT;
    void* scratch = nullptr;
    size_t bytes = 0;
    if (n_uniform == 0 && batch > 0) {
        // the varlen plan and work list go to the library-held array; uniform
        // batches need no scratch (the call is then chol_inverse_batched's)
        const hipError_t e = ci::noalloc_scratch(&scratch);
        if (e != hipSuccess) return map_err(e);
        bytes = ci::noalloc_scratch_bytes();
    }
    return chol_inverse_batched(dtype, batch, n_uniform, n_dev, offsets_dev, n_max, a, stride_a, x,
                                stride_x, opts, scratch, bytes, info, stream);
}

int chol_inverse_backward(int dtype, int64_t batch, int64_t n, const void* x, const void* g,
                          void* ga, int64_t stride, void* stream)
{
    if (!valid_dtype(dtype)) return -1;
    if (batch < 0) return -2;
    if (n < 0 || n > CI_SMALL_NMAX) return -3;
    if (batch > 0 && n > 0 && !x) return -4;
    if (batch > 0 && n > 0 && !g) return -5;
    if (batch > 0 && n > 0 && !ga) return -6;
    if (stride < n * n) return -7;
    if (batch == 0 || n == 0) return 0;
    const size_t es = elem_size(dtype);
    for (int64_t b0 = 0; b0 < batch; b0 += SMALL_CHUNK) {
        const int64_t cnt = std::min(SMALL_CHUNK, batch - b0);
        const size_t off = (size_t)(b0 * stride) * es;
        const int rc = map_err(ci::launch_backward(
            dtype, (int)n, static_cast<const char*>(x) + off, static_cast<const char*>(g) + off,
            static_cast<char*>(ga) + off, cnt, stride, (hipStream_t)stream));
        if (rc) return rc;
    }
    return 0;
}

size_t chol_workspace_size(int fn, int dtype, int64_t batch, int64_t n, const ci_opts* opts)
{
    if (!valid_dtype(dtype) || batch < 0 || n < 0) return 0;
    ci_opts o = opts ? *opts : default_opts();
    switch (fn) {
    case CI_FN_FACTOR:
        return (batch <= 1 && n > CI_SMALL_NMAX) ? ci::large_workspace(dtype, n, ci::LG_FACTOR, 0)
                                                 : 0;
    case CI_FN_INVERSE:
        return n > CI_SMALL_NMAX
                   ? ci::large_workspace(dtype, n, ci::LG_INVERSE, o.precision == CI_MIXED)
                   : 0;
    case CI_FN_BATCHED:
        return n == 0 ? ci::varlen_workspace(batch) : 0;
    case CI_FN_NONHERM: {
        // two dense batches (D D^* and its inverse), each rounded to 256 bytes
        const size_t one = ((size_t)batch * n * n * elem_size(dtype) + 255) / 256 * 256;
        return n > CI_SMALL_NMAX ? 0 : 2 * one;
    }
    default:
        return 0;
    }
}

const char* chol_status_string(int code)
{
    static thread_local char buf[96];
    if (code == 0) return "success";
    if (code == CI_ERR_UNSUPPORTED) return "unsupported combination of arguments";
    if (code == CI_ERR_WORKSPACE) return "workspace too small";
    if (code == CI_ERR_NOALLOC_LIMIT)
        return "batch larger than the library-held scratch allows (CI_NOALLOC_MAX_BATCH)";
    if (code <= CI_ERR_LAUNCH && code > CI_ERR_LAUNCH - 1000) {
        std::snprintf(buf, sizeof buf, "HIP launch error %d (%s)", CI_ERR_LAUNCH - code,
                      hipGetErrorString((hipError_t)(CI_ERR_LAUNCH - code)));
        return buf;
    }
    if (code < 0 && code > -100) {
        std::snprintf(buf, sizeof buf, "argument %d is invalid", -code);
        return buf;
    }
    return "unknown status";
}

const char* chol_version(void) { return "cholinv 0.1 (gfx950)"; }

int chol_autotune(int dtype, const ci_opts* opts, int n_lo, int n_hi, int64_t batch,
                  const char* cache_path, void* stream)
{
    if (!valid_dtype(dtype)) return -1;
    ci_opts o = opts ? *opts : default_opts();
    if (check_opts(o, dtype)) return -2;
    if (n_lo > CI_SMALL_NMAX && n_hi == n_lo) {
        if (o.method != CI_METHOD_CHOL) return -2;
        return ci::autotune_large(dtype, o.precision == CI_MIXED, o.method, o.ns_steps, n_lo,
                                  cache_path, (hipStream_t)stream);
    }
    if (n_lo < 1 || n_lo > 16) return -3;
    if (n_hi < n_lo || n_hi > 16) return -4;
    if (batch < 1) return -5;
    return ci::autotune(dtype, o.precision == CI_MIXED, o.method, o.ns_steps, n_lo, n_hi, batch,
                        cache_path, (hipStream_t)stream);
}

int chol_tuned_engine(int dtype, const ci_opts* opts, int n)
{
    if (!valid_dtype(dtype)) return -1;
    ci_opts o = opts ? *opts : default_opts();
    if (check_opts(o, dtype)) return -2;
    if (n < 0) return -3;
    const int mixed = o.precision == CI_MIXED;
    if (n == 0) return ci::tuned_varlen(dtype, mixed, o.method);
    if (n > CI_SMALL_NMAX) return ci::tuned_large(dtype, mixed, o.method, n);
    return ci::tuned_engine(dtype, mixed, o.method, n);
}

int chol_tune_set(int dtype, const ci_opts* opts, int n, int engine)
{
    if (!valid_dtype(dtype)) return -1;
    ci_opts o = opts ? *opts : default_opts();
    if (check_opts(o, dtype)) return -2;
    const int mixed = o.precision == CI_MIXED;
    if (n == 0) {
        if (engine != 0 && engine != 17 && engine != 25 && engine != 33) return -4;
        ci::tune_set_varlen(dtype, mixed, o.method, engine);
        return 0;
    }
    if (n > CI_SMALL_NMAX) {
        if (engine < 0 || engine >= ci::large_config_count()) return -4;
        ci::tune_set_large(dtype, mixed, o.method, n, engine);
        return 0;
    }
    if (n < 1 || n > 16) return -3;
    if (!ci::engine_valid(dtype, mixed, n, engine)) return -4;
    ci::tune_set(dtype, mixed, o.method, n, engine);
    return 0;
}

int chol_autotune_varlen(int dtype, const ci_opts* opts, int64_t batch, const int32_t* n_dev,
                         const int64_t* offsets_dev, int64_t n_max, const void* a, void* x,
                         void* work, size_t work_bytes, void* stream)
{
    if (!valid_dtype(dtype) || (dtype != CI_F32 && dtype != CI_F64)) return -1;
    ci_opts o = opts ? *opts : default_opts();
    if (check_opts(o, dtype)) return -2;
    if (batch < 1) return -3;
    if (!n_dev) return -4;
    if (!offsets_dev) return -5;
    if (n_max < 1 || n_max > CI_SMALL_NMAX) return -6;
    if (!a) return -7;
    if (!x || x == a) return -8;
    if (work_bytes < ci::varlen_workspace(batch) || !work) return CI_ERR_WORKSPACE;
    return ci::autotune_varlen(dtype, o.precision == CI_MIXED, o.method, o.ns_steps, batch, n_dev,
                               offsets_dev, (int)n_max, a, x, work, (hipStream_t)stream);
}

void chol_autotune_clear(void) { ci::autotune_clear(); }

}  // extern "C"
