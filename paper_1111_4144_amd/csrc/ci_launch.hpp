// ci_launch.hpp -- host-side launchers of the gfx950 kernels (internal to
// libcholinv; the public interface is include/cholinv.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ci {

enum { OP_INV = 0, OP_CHOL_FACTOR = 1, OP_LDL_FACTOR = 2 };
enum { DT_F32 = 0, DT_F64 = 1, DT_C64 = 2, DT_C128 = 3 };

// Thread-per-matrix kernels: one lane owns one whole matrix in registers.
// Compiled for orders 1..TPM_NMAX_REAL (real) and 1..TPM_NMAX_CPLX (complex);
// tpm_nmax() is the largest order dispatched to them (beyond it the register
// footprint of one matrix per lane costs more than lane groups do).
constexpr int TPM_NMAX_REAL = 16;
constexpr int TPM_NMAX_CPLX = 8;
constexpr int TPM_BLOCK = 64;

// Kernel variant request (autotuner / tests): 0 = automatic, 1 = load each
// lane's matrix directly from HBM, 2 = one-shot LDS staging, 3 = persistent
// pipelined LDS staging.
// Engine of the Newton-Schulz refinement for order 9..16 groups: the lane
// groups themselves (cross-lane broadcasts) or whole-wave MFMA products
// (environment CHOLINV_NS_ENGINE=lanes|mfma, default mfma).
enum { NS_ENGINE_MFMA = 0, NS_ENGINE_LANES = 1 };
int ns_engine();

enum { VARIANT_AUTO = 0, VARIANT_DIRECT = 1, VARIANT_STAGED = 2, VARIANT_PERSIST = 3 };

// Compute units of the current device (cached).
int device_cus();

struct BatchArgs {
    const void* a;
    void* x;
    int64_t batch, lda, sa, ldx, sx;
    int ns_steps;
    int fill;
    int32_t* info;
    void* dout;        // LDL pivots (OP_LDL_FACTOR)
    int variant = VARIANT_AUTO;
    int group = 0;     // lanes per matrix for the group kernels (0 = default)
    int ns_engine = -1;  // NS_ENGINE_* for the group kernels (-1 = process default)
};

// Engines the autotuner chooses between (orders <= 16).
enum {
    ENG_DEFAULT = 0,
    ENG_TPM_DIRECT = 1,
    ENG_TPM_STAGED = 2,
    ENG_TPM_PERSIST = 3,
    ENG_GROUP_LANES = 4,
    ENG_GROUP_MFMA = 5,
    ENG_QUAD16 = 6,
    ENG_GROUP8 = 7
};
// Recorded choice for (dtype, mixed, method, n), ENG_DEFAULT if none.
int tuned_engine(int dtype, int mixed, int method, int n);
hipError_t launch_engine(int engine, int dtype, int n, int op, int method, int mixed, BatchArgs p,
                         hipStream_t s);
// Times the candidates for orders n_lo..n_hi; returns the number of orders
// measured (>= 0) or a negative code.
int autotune(int dtype, int mixed, int method, int ns_steps, int n_lo, int n_hi, int64_t batch,
             const char* cache_path, hipStream_t s);
void autotune_clear();
// Whether `engine` can invert (dtype, mixed, order n) (ENG_DEFAULT always can),
// and recording a choice made by the caller.
bool engine_valid(int dtype, int mixed, int n, int engine);
void tune_set(int dtype, int mixed, int method, int n, int engine);
// Large orders: the recorded configuration of n's power-of-two bucket (0 =
// built-in); measuring the configurations on a test matrix of order n.
int tuned_large(int dtype, int mixed, int method, int64_t n);
void tune_set_large(int dtype, int mixed, int method, int64_t n, int cfg);
int autotune_large(int dtype, int mixed, int method, int ns_steps, int64_t n,
                   const char* cache_path, hipStream_t s);
// Uneven batches: the recorded first order of the last bucket (0 = built-in,
// 33); measuring the candidates on the caller's batch (x is overwritten).
int tuned_varlen(int dtype, int mixed, int method);
void tune_set_varlen(int dtype, int mixed, int method, int big_from);
int autotune_varlen(int dtype, int mixed, int method, int ns_steps, int64_t batch,
                    const int32_t* n_dev, const int64_t* off_dev, int n_max, const void* a, void* x,
                    void* work, hipStream_t s);

int tpm_nmax(int dtype, int mixed);

// Process-wide default variant (environment CHOLINV_TPM_VARIANT=direct|staged,
// read once; set by the tuner).
int tpm_default_variant();
void tpm_set_default_variant(int v);

// Returns a hipError_t (hipSuccess or the launch error); hipErrorNotSupported
// when no kernel exists for the combination.
hipError_t launch_tpm(int dtype, int n, int op, int method, int mixed, const BatchArgs& p,
                      hipStream_t s);
hipError_t launch_tpm_f32(int n, int op, int method, int mixed, const BatchArgs& p, hipStream_t s);
hipError_t launch_tpm_f64(int n, int op, int method, int mixed, const BatchArgs& p, hipStream_t s);
hipError_t launch_tpm_c64(int n, int op, int method, int mixed, const BatchArgs& p, hipStream_t s);
hipError_t launch_tpm_c128(int n, int op, int method, int mixed, const BatchArgs& p, hipStream_t s);

// Group-per-matrix kernels (orders above tpm_nmax, up to 64 for real and 32
// for complex elements).
hipError_t launch_group(int dtype, int n, int op, int method, int mixed, const BatchArgs& p,
                        hipStream_t s);
hipError_t launch_group_f32(int n, int op, int method, int mixed, const BatchArgs& p, hipStream_t s);
hipError_t launch_group_f64(int n, int op, int method, int mixed, const BatchArgs& p, hipStream_t s);
hipError_t launch_group_c64(int n, int op, int method, int mixed, const BatchArgs& p, hipStream_t s);
hipError_t launch_group_c128(int n, int op, int method, int mixed, const BatchArgs& p, hipStream_t s);
// Four lanes per matrix, sixteen matrices per wave (orders <= 16, float and
// complex float, inversion only; mixed precision refines on MFMA).
// Eight lanes per matrix (orders <= 16, double and complex double, plain
// precision, inversion only).
hipError_t launch_group8(int dtype, int n, int op, int method, int mixed, const BatchArgs& p,
                         hipStream_t s);
hipError_t launch_quad16(int dtype, int n, int op, int method, int mixed, const BatchArgs& p,
                         hipStream_t s);
// LDS-resident group kernels for orders 17..64 (real) / 17..32 (complex).
hipError_t launch_wpm_f32(int n, int op, int method, int mixed, const BatchArgs& p, hipStream_t s);
hipError_t launch_wpm_f64(int n, int op, int method, int mixed, const BatchArgs& p, hipStream_t s);
hipError_t launch_wpm_c64(int n, int op, int method, int mixed, const BatchArgs& p, hipStream_t s);
hipError_t launch_wpm_c128(int n, int op, int method, int mixed, const BatchArgs& p, hipStream_t s);

// Solves A x = y with the factor of A (orders <= 64): one lane per
// right-hand side.  Right-hand sides are the columns of an n x nrhs row-major
// block per matrix; d holds the LDL pivots (real type of V, n per matrix).
struct SolveArgs {
    const void* r;
    int64_t ldr, sr;
    const void* d;
    const void* b;
    int64_t ldb, sb;
    void* x;
    int64_t ldx, sx;
    int64_t batch;
    int n, nrhs;
};
hipError_t launch_solve(int dtype, int method, const SolveArgs& p, hipStream_t s);

// Backward gA = -X Gh X.
hipError_t launch_backward(int dtype, int n, const void* x, const void* g, void* ga,
                           int64_t batch, int64_t stride, hipStream_t s);

}  // namespace ci
