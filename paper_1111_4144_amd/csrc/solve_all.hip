// solve_all.hip -- batched linear solves A x = y with the factor of A.
//
// Cholesky (Section II, eqs. 5-7): R^* b = y by forward substitution, then
// R x = b by back substitution.  LDL (Section II.A, eqs. 12-14): R^* c = y
// with the unit R, b_i = c_i / d_i, then R x = b.  Each right-hand side costs
// n^2/2 multiplies per substitution.
//
// One lane solves one right-hand side of one matrix.  Orders up to 16 keep
// the vector in registers (loops unrolled to a compile-time bound, the order
// itself a runtime value); orders 17..64 keep it in LDS, one column per lane
// at a lane-interleaved address so a wave's accesses fall in distinct banks.
// Dense batches with one right-hand side (the factors back to back, each
// vector contiguous) take the staged kernel: a block of 64 lanes copies its 64
// factors into LDS with 16-byte loads (upper triangles kept, packed), loads
// each vector with wide loads, and each lane substitutes from its LDS slot.
// Other layouts read the factor from global memory entry by entry.
#include "ci_launch.hpp"
#include "ci_types.hpp"
#include "cholinv.h"
#include "tpm_impl.hpp"

namespace ci {

namespace {

constexpr int SOLVE_THREADS = 256;

template <class V, int METHOD, int NMAX>
__global__ void __launch_bounds__(SOLVE_THREADS) k_solve_reg(SolveArgs p)
{
    using R = typename vt<V>::real;
    const int64_t t = (int64_t)blockIdx.x * SOLVE_THREADS + threadIdx.x;
    if (t >= p.batch * p.nrhs) return;
    const int64_t m = t / p.nrhs;
    const int64_t c = t - m * p.nrhs;
    const int n = p.n;
    const V* __restrict__ r = (const V*)p.r + m * p.sr;
    const V* __restrict__ b = (const V*)p.b + m * p.sb + c;
    V* __restrict__ x = (V*)p.x + m * p.sx + c;
    const R* __restrict__ dv = (const R*)p.d + m * n;

    V y[NMAX];
    R inv[NMAX];
#pragma unroll
    for (int i = 0; i < NMAX; ++i) y[i] = (i < n) ? b[(int64_t)i * p.ldb] : mk<V>(R(0));

    // forward substitution with R^*: column i of R above the diagonal
#pragma unroll
    for (int i = 0; i < NMAX; ++i) {
        if (i < n) {
            V acc = y[i];
#pragma unroll
            for (int k = 0; k < i; ++k) msubc(acc, r[(int64_t)k * p.ldr + i], y[k]);
            if constexpr (METHOD == 0) {
                inv[i] = R(1) / re(r[(int64_t)i * p.ldr + i]);
                y[i] = scal(acc, inv[i]);            // b_i
            } else {
                inv[i] = R(1) / dv[i];
                y[i] = acc;                          // c_i (unit R: no division)
            }
        }
    }
    // back substitution with R: row i of R right of the diagonal
#pragma unroll
    for (int i = NMAX - 1; i >= 0; --i) {
        if (i < n) {
            V acc = (METHOD == 0) ? y[i] : scal(y[i], inv[i]);    // LDL: b_i = c_i / d_i
#pragma unroll
            for (int k = i + 1; k < NMAX; ++k)
                if (k < n) msub(acc, r[(int64_t)i * p.ldr + k], y[k]);
            y[i] = (METHOD == 0) ? scal(acc, inv[i]) : acc;
        }
    }
#pragma unroll
    for (int i = 0; i < NMAX; ++i)
        if (i < n) x[(int64_t)i * p.ldx] = y[i];
}

// 64-bit complex vectors of order 64 take 64 KB for a 64-lane block; the
// 16-byte type runs 32 lanes per block to keep the block's LDS at 32 KB.
template <class V> constexpr int LDS_LANES = sizeof(V) == 16 ? 32 : 64;

template <class V, int METHOD>
__global__ void __launch_bounds__(LDS_LANES<V>) k_solve_lds(SolveArgs p)
{
    using R = typename vt<V>::real;
    constexpr int L = LDS_LANES<V>;
    __shared__ V ys[CI_SMALL_NMAX * L];
    const int lane = threadIdx.x;
    const int64_t t = (int64_t)blockIdx.x * L + lane;
    if (t >= p.batch * p.nrhs) return;            // lanes never share LDS entries
    const int64_t m = t / p.nrhs;
    const int64_t c = t - m * p.nrhs;
    const int n = p.n;
    const V* __restrict__ r = (const V*)p.r + m * p.sr;
    const V* __restrict__ b = (const V*)p.b + m * p.sb + c;
    V* __restrict__ x = (V*)p.x + m * p.sx + c;
    const R* __restrict__ dv = (const R*)p.d + m * n;
    V* y = ys + lane;                              // y[k * L] is entry k

    for (int i = 0; i < n; ++i) y[i * L] = b[(int64_t)i * p.ldb];
    for (int i = 0; i < n; ++i) {
        V acc = y[i * L];
        for (int k = 0; k < i; ++k) msubc(acc, r[(int64_t)k * p.ldr + i], y[k * L]);
        if constexpr (METHOD == 0) acc = scal(acc, R(1) / re(r[(int64_t)i * p.ldr + i]));
        y[i * L] = acc;                            // CHOL: b_i; LDL: c_i
    }
    for (int i = n - 1; i >= 0; --i) {
        V acc = y[i * L];
        if constexpr (METHOD == 1) acc = scal(acc, R(1) / dv[i]);   // b_i = c_i / d_i
        const V* ri = r + (int64_t)i * p.ldr;
        for (int k = i + 1; k < n; ++k) msub(acc, ri[k], y[k * L]);
        if constexpr (METHOD == 0) acc = scal(acc, R(1) / re(ri[i]));
        y[i * L] = acc;
    }
    for (int i = 0; i < n; ++i) x[(int64_t)i * p.ldx] = y[i * L];
}

// Exact order N, one right-hand side, dense: factor from its packed LDS slot.
template <class V, int METHOD, int N>
__global__ void __launch_bounds__(TPM_BLOCK) k_solve_staged(SolveArgs p)
{
    using R = typename vt<V>::real;
    constexpr int SL = Slot<N, true>::SIZE;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    V* sm = reinterpret_cast<V*>(smem_raw);
    const int t = threadIdx.x;
    const int64_t b0 = (int64_t)blockIdx.x * TPM_BLOCK;
    const int nvalid = (int)((p.batch - b0) < TPM_BLOCK ? (p.batch - b0) : TPM_BLOCK);
    stage_in<V, N, true>((const V*)p.r, sm, b0, nvalid, t);
    __syncthreads();
    if (t >= nvalid) return;
    const int64_t m = b0 + t;
    const V* slot = sm + t * SL;
    V y[N];
    load_vec<V, N>((const V*)p.b + m * N, y);
    R inv[N];
#pragma unroll
    for (int i = 0; i < N; ++i) {
        V acc = y[i];
#pragma unroll
        for (int k = 0; k < i; ++k) msubc(acc, slot[pidx<N>(k, i)], y[k]);
        if constexpr (METHOD == 0) {
            inv[i] = R(1) / re(slot[pidx<N>(i, i)]);
            y[i] = scal(acc, inv[i]);
        } else {
            inv[i] = R(1) / ((const R*)p.d)[m * N + i];
            y[i] = acc;
        }
    }
#pragma unroll
    for (int i = N - 1; i >= 0; --i) {
        V acc = (METHOD == 0) ? y[i] : scal(y[i], inv[i]);
#pragma unroll
        for (int k = i + 1; k < N; ++k) msub(acc, slot[pidx<N>(i, k)], y[k]);
        y[i] = (METHOD == 0) ? scal(acc, inv[i]) : acc;
    }
    store_vec<V, N>((V*)p.x + m * N, y);
}

template <class V, int METHOD, int N>
hipError_t solve_staged(const SolveArgs& p, hipStream_t s)
{
    const size_t smem = (size_t)TPM_BLOCK * Slot<N, true>::SIZE * sizeof(V);
    auto kern = k_solve_staged<V, METHOD, N>;
    if (smem > 65536) {
        static bool once = false;
        if (!once) {
            hipError_t e = hipFuncSetAttribute((const void*)kern,
                                               hipFuncAttributeMaxDynamicSharedMemorySize,
                                               (int)smem);
            if (e != hipSuccess) return e;
            once = true;
        }
    }
    const int64_t blocks = (p.batch + TPM_BLOCK - 1) / TPM_BLOCK;
    hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(TPM_BLOCK), smem, s, p);
    return hipGetLastError();
}

// The staged kernel needs whole factors back to back, contiguous vectors and
// 16-byte aligned bases (its wide accesses).
bool staged_layout(const SolveArgs& p, size_t es)
{
    const int64_t n = p.n;
    const bool dense = p.nrhs == 1 && p.ldr == n && (p.batch == 1 || p.sr == n * n) &&
                       p.ldb == 1 && p.ldx == 1 && (p.batch == 1 || (p.sb == n && p.sx == n));
    const auto al = [](const void* q) { return ((uintptr_t)q & 15) == 0; };
    return dense && al(p.r) && al(p.b) && al(p.x) && (n * es) % 16 == 0;
}

template <class V, int METHOD>
hipError_t solve_method(const SolveArgs& p, hipStream_t s)
{
    const int64_t lanes = p.batch * p.nrhs;
    if (staged_layout(p, sizeof(V))) {
        switch (p.n) {
        case 2: return solve_staged<V, METHOD, 2>(p, s);
        case 4: return solve_staged<V, METHOD, 4>(p, s);
        case 8: return solve_staged<V, METHOD, 8>(p, s);
        case 16: return solve_staged<V, METHOD, 16>(p, s);
        default: break;
        }
    }
    if (p.n > 16) {
        constexpr int L = LDS_LANES<V>;
        hipLaunchKernelGGL((k_solve_lds<V, METHOD>), dim3((unsigned)((lanes + L - 1) / L)),
                           dim3(L), 0, s, p);
        return hipGetLastError();
    }
    const dim3 grid((unsigned)((lanes + SOLVE_THREADS - 1) / SOLVE_THREADS)), block(SOLVE_THREADS);
    if (p.n <= 4) hipLaunchKernelGGL((k_solve_reg<V, METHOD, 4>), grid, block, 0, s, p);
    else if (p.n <= 8) hipLaunchKernelGGL((k_solve_reg<V, METHOD, 8>), grid, block, 0, s, p);
    else hipLaunchKernelGGL((k_solve_reg<V, METHOD, 16>), grid, block, 0, s, p);
    return hipGetLastError();
}

template <class V>
hipError_t solve_type(int method, const SolveArgs& p, hipStream_t s)
{
    return method == 0 ? solve_method<V, 0>(p, s) : solve_method<V, 1>(p, s);
}

}  // namespace

hipError_t launch_solve(int dtype, int method, const SolveArgs& p, hipStream_t s)
{
    if (p.batch <= 0 || p.n <= 0 || p.nrhs <= 0) return hipSuccess;
    if (p.n > CI_SMALL_NMAX) return hipErrorNotSupported;
    switch (dtype) {
    case DT_F32: return solve_type<float>(method, p, s);
    case DT_F64: return solve_type<double>(method, p, s);
    case DT_C64: return solve_type<cf>(method, p, s);
    case DT_C128: return solve_type<cd>(method, p, s);
    default: return hipErrorNotSupported;
    }
}

}  // namespace ci
