// tune.hip -- the autotuner of the small-order engines.
//
// For orders up to 16 several kernels can invert a batch: the one-lane-per-
// matrix kernels with direct loads, one-shot LDS staging or persistent
// staging (orders up to the per-type register limit), the 16-lane group
// kernels with the Newton-Schulz step on the lane groups or on MFMA (mixed
// precision), the 4-lane groups with sixteen matrices per wave (orders
// 9..16, float and complex float) and the 8-lane groups of the FP64 types
// (plain precision).  chol_autotune times every candidate for each order of a range
// on a synthetic batch on the caller's device and stream and records the
// fastest; run_small consults the record.  Choices can be persisted in a text
// cache keyed by the device (name and compute-unit count), so later processes
// load them instead of measuring.  Ties within 1% go to the lower engine
// number, so the choice is reproducible.
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>

#include "ci_large.hpp"
#include "ci_launch.hpp"
#include "ci_types.hpp"
#include "cholinv.h"

namespace ci {

namespace {

std::mutex g_mu;
// [dtype][mixed][method][n] -> engine (0 = built-in default)
int g_table[4][2][2][65];
// large orders: [dtype][mixed][method][floor(log2 n)] -> configuration index
int g_large[4][2][2][32];
// uneven batches: [dtype][mixed][method] -> first order of the last bucket (0 = 33)
int g_varlen[4][2][2];

int log2_bucket(int64_t n)
{
    int b = 0;
    while (b < 31 && ((int64_t)2 << b) <= n) ++b;
    return b;
}

std::string device_key()
{
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
        return "unknown";
    std::string name = prop.gcnArchName;
    for (char& c : name)
        if (c == ' ') c = '_';
    return name + ":" + std::to_string(prop.multiProcessorCount);
}

// Diagonally dominant Hermitian matrices: a_ii = n + 1, a_ij = 1/(1 + i + j)
// (+ an imaginary part (j - i)/(8 n) above the diagonal for complex types).
template <class V>
__global__ void k_tune_fill(V* a, int64_t batch, int n)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= batch * n * n) return;
    const int i = (int)((e / n) % n), j = (int)(e % n);
    using R = typename vt<V>::real;
    const R re = (i == j) ? R(n + 1) : R(1) / R(1 + i + j);
    V v = mk<V>(re);
    if constexpr (vt<V>::cplx) {
        if (i != j) v.im = (j > i ? R(1) : R(-1)) * R(j > i ? j - i : i - j) / R(8 * n);
    }
    a[e] = v;
}

hipError_t fill(int dtype, void* a, int64_t batch, int n, hipStream_t s)
{
    const unsigned blocks = (unsigned)((batch * n * n + 255) / 256);
    switch (dtype) {
    case DT_F32: hipLaunchKernelGGL(k_tune_fill<float>, dim3(blocks), dim3(256), 0, s, (float*)a, batch, n); break;
    case DT_F64: hipLaunchKernelGGL(k_tune_fill<double>, dim3(blocks), dim3(256), 0, s, (double*)a, batch, n); break;
    case DT_C64: hipLaunchKernelGGL(k_tune_fill<cf>, dim3(blocks), dim3(256), 0, s, (cf*)a, batch, n); break;
    default: hipLaunchKernelGGL(k_tune_fill<cd>, dim3(blocks), dim3(256), 0, s, (cd*)a, batch, n); break;
    }
    return hipGetLastError();
}

size_t elem_size(int dtype) { return dtype == DT_F32 ? 4 : (dtype == DT_C128 ? 16 : 8); }

// Candidates for (dtype, mixed, n), in engine order.
int candidates(int dtype, int mixed, int n, int* out)
{
    int k = 0;
    if (n <= tpm_nmax(dtype, mixed)) {
        out[k++] = ENG_TPM_DIRECT;
        out[k++] = ENG_TPM_STAGED;
        out[k++] = ENG_TPM_PERSIST;
    }
    if (n <= 16) {
        out[k++] = ENG_GROUP_LANES;
        if (mixed && (dtype == DT_F32 || dtype == DT_C64)) out[k++] = ENG_GROUP_MFMA;
        if (n >= 9 && (dtype == DT_F32 || dtype == DT_C64)) out[k++] = ENG_QUAD16;
        if (!mixed && (dtype == DT_F64 || dtype == DT_C128)) out[k++] = ENG_GROUP8;
    }
    return k;
}

// Cache lines: "cholinv-tune v1 <device> dtype mixed method n choice us"; n in
// 1..16 records an engine, n > 64 a large-order configuration (for the
// order's power-of-two bucket), n = 0 the uneven-batch bucket edge.
bool load_cache(const char* path, const std::string& dev, int dtype, int mixed, int method,
                int n_lo, int n_hi, bool* have)
{
    FILE* f = std::fopen(path, "r");
    if (!f) return false;
    char line[512];
    while (std::fgets(line, sizeof line, f)) {
        char dname[256];
        int d, p, m, n, e;
        double us;
        if (std::sscanf(line, "cholinv-tune v1 %255s %d %d %d %d %d %lf", dname, &d, &p, &m, &n,
                        &e, &us) != 7)
            continue;
        if (dev != dname || d != dtype || p != mixed || m != method || n < n_lo || n > n_hi)
            continue;
        if (n > 64) {
            if (e < 0 || e >= large_config_count()) continue;
            g_large[dtype][mixed][method][log2_bucket(n)] = e;
            have[0] = true;
            continue;
        }
        if (e < ENG_DEFAULT || e > ENG_GROUP8) continue;
        g_table[dtype][mixed][method][n] = e;
        have[n] = true;
    }
    std::fclose(f);
    return true;
}

}  // namespace

int tuned_engine(int dtype, int mixed, int method, int n)
{
    if (dtype < 0 || dtype > 3 || n < 0 || n > 64) return ENG_DEFAULT;
    std::lock_guard<std::mutex> lk(g_mu);
    return g_table[dtype][mixed ? 1 : 0][method ? 1 : 0][n];
}

// Launch one candidate engine on a uniform dense batch.
hipError_t launch_engine(int engine, int dtype, int n, int op, int method, int mixed, BatchArgs p,
                         hipStream_t s)
{
    switch (engine) {
    case ENG_TPM_DIRECT: p.variant = VARIANT_DIRECT; return launch_tpm(dtype, n, op, method, mixed, p, s);
    case ENG_TPM_STAGED: p.variant = VARIANT_STAGED; return launch_tpm(dtype, n, op, method, mixed, p, s);
    case ENG_TPM_PERSIST: p.variant = VARIANT_PERSIST; return launch_tpm(dtype, n, op, method, mixed, p, s);
    case ENG_GROUP_LANES: p.ns_engine = NS_ENGINE_LANES; return launch_group(dtype, n, op, method, mixed, p, s);
    case ENG_GROUP_MFMA: p.ns_engine = NS_ENGINE_MFMA; return launch_group(dtype, n, op, method, mixed, p, s);
    case ENG_QUAD16: return launch_quad16(dtype, n, op, method, mixed, p, s);
    case ENG_GROUP8: return launch_group8(dtype, n, op, method, mixed, p, s);
    default: return hipErrorInvalidValue;
    }
}

int autotune(int dtype, int mixed, int method, int ns_steps, int n_lo, int n_hi, int64_t batch,
             const char* cache_path, hipStream_t s)
{
    const std::string dev = device_key();
    bool have[65] = {false};
    if (cache_path) {
        std::lock_guard<std::mutex> lk(g_mu);
        load_cache(cache_path, dev, dtype, mixed, method, n_lo, n_hi, have);
    }
    const size_t es = elem_size(dtype);
    void *a = nullptr, *x = nullptr, *info = nullptr;
    const size_t bytes = (size_t)batch * n_hi * n_hi * es;
    if (hipMalloc(&a, bytes) != hipSuccess) return -1000 - (int)hipErrorOutOfMemory;
    if (hipMalloc(&x, bytes) != hipSuccess) { (void)hipFree(a); return -1000 - (int)hipErrorOutOfMemory; }
    if (hipMalloc(&info, (size_t)batch * 4) != hipSuccess) {
        (void)hipFree(a); (void)hipFree(x);
        return -1000 - (int)hipErrorOutOfMemory;
    }
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    int measured = 0;
    hipError_t err = hipSuccess;
    FILE* out = cache_path ? std::fopen(cache_path, "a") : nullptr;
    for (int n = n_lo; n <= n_hi && err == hipSuccess; ++n) {
        if (have[n]) continue;
        int cand[8];
        const int nc = candidates(dtype, mixed, n, cand);
        if (nc < 2) continue;                      // nothing to choose
        err = fill(dtype, a, batch, n, s);
        BatchArgs p{a, x, batch, n, (int64_t)n * n, n, (int64_t)n * n, ns_steps, 1,
                    (int32_t*)info, nullptr};
        int best = ENG_DEFAULT;
        float best_ms = 0.f;
        for (int c = 0; c < nc && err == hipSuccess; ++c) {
            err = launch_engine(cand[c], dtype, n, OP_INV, method, mixed, p, s);   // warm-up
            if (err != hipSuccess) break;
            (void)hipEventRecord(e0, s);
            for (int r = 0; r < 3 && err == hipSuccess; ++r)
                err = launch_engine(cand[c], dtype, n, OP_INV, method, mixed, p, s);
            (void)hipEventRecord(e1, s);
            if (err != hipSuccess) break;
            err = hipEventSynchronize(e1);
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            if (best == ENG_DEFAULT || ms < best_ms * 0.99f) {
                best = cand[c];
                best_ms = ms;
            }
        }
        if (err != hipSuccess) break;
        {
            std::lock_guard<std::mutex> lk(g_mu);
            g_table[dtype][mixed][method][n] = best;
        }
        if (out)
            std::fprintf(out, "cholinv-tune v1 %s %d %d %d %d %d %.3f\n", dev.c_str(), dtype, mixed,
                         method, n, best, 1e3 * best_ms / 3);
        ++measured;
    }
    if (out) std::fclose(out);
    (void)hipStreamSynchronize(s);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(a);
    (void)hipFree(x);
    (void)hipFree(info);
    return err == hipSuccess ? measured : -1000 - (int)err;
}

bool engine_valid(int dtype, int mixed, int n, int engine)
{
    if (engine == ENG_DEFAULT) return true;
    int cand[8];
    const int nc = candidates(dtype, mixed, n, cand);
    for (int c = 0; c < nc; ++c)
        if (cand[c] == engine) return true;
    return false;
}

void tune_set(int dtype, int mixed, int method, int n, int engine)
{
    std::lock_guard<std::mutex> lk(g_mu);
    g_table[dtype][mixed ? 1 : 0][method ? 1 : 0][n] = engine;
}

void autotune_clear()
{
    std::lock_guard<std::mutex> lk(g_mu);
    std::memset(g_table, 0, sizeof g_table);
    std::memset(g_large, 0, sizeof g_large);
    std::memset(g_varlen, 0, sizeof g_varlen);
}

// ---- large orders ---------------------------------------------------------------
int tuned_large(int dtype, int mixed, int method, int64_t n)
{
    if (dtype < 0 || dtype > 3) return 0;
    std::lock_guard<std::mutex> lk(g_mu);
    return g_large[dtype][mixed ? 1 : 0][method ? 1 : 0][log2_bucket(n)];
}

void tune_set_large(int dtype, int mixed, int method, int64_t n, int cfg)
{
    std::lock_guard<std::mutex> lk(g_mu);
    g_large[dtype][mixed ? 1 : 0][method ? 1 : 0][log2_bucket(n)] = cfg;
}

namespace {
// symmetric positive definite test matrix a_ij = 1/(1 + |i - j|) + n [i == j]
template <class T>
__global__ void k_tune_spd(T* a, int64_t n)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * n) return;
    const int64_t i = e / n, j = e % n, d = i > j ? i - j : j - i;
    a[e] = T(1) / T(1 + d) + (i == j ? T(n) : T(0));
}
}  // namespace

int autotune_large(int dtype, int mixed, int method, int ns_steps, int64_t n, const char* cache_path,
                   hipStream_t s)
{
    if (dtype != DT_F32 && dtype != DT_F64) return -1000 - (int)hipErrorNotSupported;
    const std::string dev = device_key();
    bool have[65] = {false};
    if (cache_path) {
        std::lock_guard<std::mutex> lk(g_mu);
        load_cache(cache_path, dev, dtype, mixed, method, (int)n, (int)n, have);
        if (have[0]) return 0;
    }
    const size_t es = dtype == DT_F32 ? 4 : 8, bytes = (size_t)n * n * es;
    const size_t wbytes = large_workspace(dtype, n, LG_INVERSE, mixed);
    void *a = nullptr, *x = nullptr, *w = nullptr;
    if (hipMalloc(&a, bytes) != hipSuccess) return -1000 - (int)hipErrorOutOfMemory;
    if (hipMalloc(&x, bytes) != hipSuccess) { (void)hipFree(a); return -1000 - (int)hipErrorOutOfMemory; }
    if (hipMalloc(&w, wbytes) != hipSuccess) {
        (void)hipFree(a); (void)hipFree(x);
        return -1000 - (int)hipErrorOutOfMemory;
    }
    const unsigned blocks = (unsigned)((n * n + 255) / 256);
    if (dtype == DT_F32) hipLaunchKernelGGL(k_tune_spd<float>, dim3(blocks), dim3(256), 0, s, (float*)a, n);
    else hipLaunchKernelGGL(k_tune_spd<double>, dim3(blocks), dim3(256), 0, s, (double*)a, n);
    hipError_t err = hipGetLastError();
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    int best = 0;
    float best_ms = 0.f;
    for (int c = 0; c < large_config_count() && err == hipSuccess; ++c) {
        err = large_inverse(dtype, n, a, n, x, n, mixed, ns_steps, 1, nullptr, w, s, c);  // warm-up
        if (err != hipSuccess) break;
        (void)hipEventRecord(e0, s);
        for (int r = 0; r < 2 && err == hipSuccess; ++r)
            err = large_inverse(dtype, n, a, n, x, n, mixed, ns_steps, 1, nullptr, w, s, c);
        (void)hipEventRecord(e1, s);
        if (err != hipSuccess) break;
        err = hipEventSynchronize(e1);
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        if (c == 0 || ms < best_ms * 0.99f) {
            best = c;
            best_ms = ms;
        }
    }
    if (err == hipSuccess) {
        tune_set_large(dtype, mixed, method, n, best);
        FILE* out = cache_path ? std::fopen(cache_path, "a") : nullptr;
        if (out) {
            std::fprintf(out, "cholinv-tune v1 %s %d %d %d %lld %d %.3f\n", dev.c_str(), dtype, mixed,
                         method, (long long)n, best, 1e3 * best_ms / 2);
            std::fclose(out);
        }
    }
    (void)hipStreamSynchronize(s);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(a);
    (void)hipFree(x);
    (void)hipFree(w);
    return err == hipSuccess ? 1 : -1000 - (int)err;
}

// ---- uneven batches ---------------------------------------------------------------
int tuned_varlen(int dtype, int mixed, int method)
{
    if (dtype < 0 || dtype > 3) return 0;
    std::lock_guard<std::mutex> lk(g_mu);
    return g_varlen[dtype][mixed ? 1 : 0][method ? 1 : 0];
}

void tune_set_varlen(int dtype, int mixed, int method, int big_from)
{
    std::lock_guard<std::mutex> lk(g_mu);
    g_varlen[dtype][mixed ? 1 : 0][method ? 1 : 0] = big_from;
}

int autotune_varlen(int dtype, int mixed, int method, int ns_steps, int64_t batch,
                    const int32_t* n_dev, const int64_t* off_dev, int n_max, const void* a, void* x,
                    void* work, hipStream_t s)
{
    static const int cand[] = {33, 25, 17};
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    hipError_t err = hipSuccess;
    int best = 33;
    float best_ms = 0.f;
    for (int c = 0; c < 3 && err == hipSuccess; ++c) {
        err = launch_varlen(dtype, batch, n_dev, off_dev, n_max, a, x, method, mixed, ns_steps, 1,
                            nullptr, work, s, cand[c]);                              // warm-up
        if (err != hipSuccess) break;
        (void)hipEventRecord(e0, s);
        for (int r = 0; r < 3 && err == hipSuccess; ++r)
            err = launch_varlen(dtype, batch, n_dev, off_dev, n_max, a, x, method, mixed, ns_steps,
                                1, nullptr, work, s, cand[c]);
        (void)hipEventRecord(e1, s);
        if (err != hipSuccess) break;
        err = hipEventSynchronize(e1);
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        if (c == 0 || ms < best_ms * 0.99f) {
            best = cand[c];
            best_ms = ms;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (err != hipSuccess) return -1000 - (int)err;
    tune_set_varlen(dtype, mixed, method, best);
    return best;
}

}  // namespace ci
