// varlen_impl.hpp -- one persistent launch for a packed batch of matrices of
// uneven orders (1..64).  Included by one translation unit per element type.
//
// Device-side prologue (no host synchronisation, capturable in a HIP graph):
//   1. count   histogram of the orders;
//   2. scan    orders are laid out largest first: per order n its first item
//              in the sorted index list and its tile range;
//   3. scatter every matrix index into the sorted list.
// Tiles: an order n <= 8 tile is up to 64 matrices (one lane each, registers);
// 9..16 up to 4 matrices (16-lane groups padded to 16 with the identity,
// which leaves the n x n block exact); 17..32 up to 2 (LDS-resident, one lane
// per column) and 33..64 one matrix (LDS-resident, four lanes per column,
// four waves).  The edge of the last bucket (33) can move down to 25 or 17
// (a tuned choice): those orders then take whole four-wave blocks.  Two
// persistent kernels, one per block shape, take tiles from their own atomic
// counters until none are left (every wave reaches that exit): first the
// last bucket, then the rest, largest orders first within each.  Results do
// not depend on which wave takes which tile.
#pragma once

#include "group_impl.hpp"
#include "leaf_impl.hpp"
#include "tpm_impl.hpp"
#include "wpm_impl.hpp"

namespace ci {

struct VarlenPlan {
    int next;              // tile counter of the orders <= 32 kernel (starts at nbig)
    int ntiles;
    int next_big;          // tile counter of the last bucket's kernel (starts at 0)
    int nbig;              // tiles of orders big_from..64 (one matrix each, first in the order)
    int big_from;          // smallest order of the four-waves-per-matrix kernel (17, 25 or 33)
    int count[65];         // matrices per order
    int item_start[65];    // first position of order n in the sorted list
    int tile_start[65];    // tile range of order n: [tile_start, tile_end)
    int tile_end[65];
    int cursor[65];        // scatter cursors
};

CI_D int vl_tile_size(int n) { return n <= 8 ? 64 : n <= 16 ? 4 : n <= 32 ? 2 : 1; }

__global__ void k_vl_init(VarlenPlan* plan)
{
    int* p = reinterpret_cast<int*>(plan);
    for (int i = threadIdx.x; i < (int)(sizeof(VarlenPlan) / sizeof(int)); i += blockDim.x) p[i] = 0;
}

// Orders are counted per block in LDS first, so each block adds to a global
// counter once per order present instead of once per matrix.
__global__ void __launch_bounds__(256)
k_vl_count(const int32_t* __restrict__ ns, int64_t batch, int nmax, VarlenPlan* plan,
           int32_t* __restrict__ info)
{
    __shared__ int local[65];
    for (int t = threadIdx.x; t < 65; t += blockDim.x) local[t] = 0;
    __syncthreads();
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b < batch) {
        const int n = ns[b];
        if (n < 0 || n > nmax) {
            if (info) info[b] = -1;
        } else if (n == 0) {
            if (info) info[b] = 0;
        } else {
            atomicAdd(&local[n], 1);
        }
    }
    __syncthreads();
    for (int t = threadIdx.x; t < 65; t += blockDim.x)
        if (local[t]) atomicAdd(&plan->count[t], local[t]);
}

__global__ void k_vl_scan(VarlenPlan* plan, int big_from)
{
    if (threadIdx.x != 0) return;
    int items = 0, tiles = 0;
    plan->big_from = big_from;
    for (int n = 64; n >= 1; --n) {
        const int c = plan->count[n];
        const int ts = n >= big_from ? 1 : vl_tile_size(n);
        plan->item_start[n] = items;
        plan->tile_start[n] = tiles;
        tiles += (c + ts - 1) / ts;
        plan->tile_end[n] = tiles;
        items += c;
    }
    plan->ntiles = tiles;
    plan->nbig = plan->tile_end[big_from];
    plan->next = plan->nbig;
    plan->next_big = 0;
}

// Each block reserves one contiguous range per order with a single global
// atomic and places its matrices inside it with LDS atomics.  The order of
// matrices within an order's range is therefore not the batch order; results
// do not depend on it.
__global__ void __launch_bounds__(256)
k_vl_scatter(const int32_t* __restrict__ ns, int64_t batch, int nmax, VarlenPlan* plan,
             int32_t* __restrict__ sorted)
{
    __shared__ int local[65], base[65];
    for (int t = threadIdx.x; t < 65; t += blockDim.x) local[t] = 0;
    __syncthreads();
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int n = 0, slot = -1;
    if (b < batch) {
        n = ns[b];
        if (n >= 1 && n <= nmax) slot = atomicAdd(&local[n], 1);
    }
    __syncthreads();
    for (int t = threadIdx.x; t < 65; t += blockDim.x)
        if (local[t]) base[t] = plan->item_start[t] + atomicAdd(&plan->cursor[t], local[t]);
    __syncthreads();
    if (slot >= 0) sorted[base[n] + slot] = (int32_t)b;
}

// One lane, one matrix of order N (dense, leading dimension N).
template <class V, int N, int METHOD, int MIXED>
CI_D int vl_lane(const V* __restrict__ a, V* x, int ns_steps, int fill)
{
    V A[N][N];
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
        for (int j = i; j < N; ++j) A[i][j] = a[i * N + j];
    return tpm_body<V, N, OP_INV, METHOD, MIXED>(A, OutDense<V>{x, N, fill != 0}, ns_steps, false,
                                                 nullptr, nullptr);
}

template <class V, int METHOD, int MIXED>
__global__ void __launch_bounds__(64)
k_varlen(const V* __restrict__ a, V* x, const int64_t* __restrict__ offs,
         const int32_t* __restrict__ sorted, VarlenPlan* plan, int ns_steps, int fill,
         int32_t* __restrict__ info)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ int s_tile;
    const int lane = threadIdx.x;
    for (;;) {
        if (lane == 0) s_tile = atomicAdd(&plan->next, 1);
        __syncthreads();
        const int t = s_tile;
        __syncthreads();
        if (t >= plan->ntiles) break;
        int n = 64;
        while (n > 1 && t >= plan->tile_end[n]) --n;
        const int per = vl_tile_size(n);
        const int k = t - plan->tile_start[n];
        const int first = plan->item_start[n] + k * per;
        const int cnt = min(per, plan->count[n] - k * per);
        if (n <= 8) {
            if (lane < cnt) {
                const int b = sorted[first + lane];
                const int64_t o = offs[b];
                int f = 0;
                switch (n) {
                case 1: f = vl_lane<V, 1, METHOD, MIXED>(a + o, x + o, ns_steps, fill); break;
                case 2: f = vl_lane<V, 2, METHOD, MIXED>(a + o, x + o, ns_steps, fill); break;
                case 3: f = vl_lane<V, 3, METHOD, MIXED>(a + o, x + o, ns_steps, fill); break;
                case 4: f = vl_lane<V, 4, METHOD, MIXED>(a + o, x + o, ns_steps, fill); break;
                case 5: f = vl_lane<V, 5, METHOD, MIXED>(a + o, x + o, ns_steps, fill); break;
                case 6: f = vl_lane<V, 6, METHOD, MIXED>(a + o, x + o, ns_steps, fill); break;
                case 7: f = vl_lane<V, 7, METHOD, MIXED>(a + o, x + o, ns_steps, fill); break;
                default: f = vl_lane<V, 8, METHOD, MIXED>(a + o, x + o, ns_steps, fill); break;
                }
                if (info) info[b] = f;
            }
        } else if (n <= 16) {
            const int g = lane / 16;
            const bool valid = g < cnt;
            const int b = sorted[first + (valid ? g : 0)];
            const int64_t o = offs[b];
            group_matrix<V, 16, 16, OP_INV, METHOD, MIXED>(a + o, n, n, x + o, n, valid, fill,
                                                           ns_steps, lane % 16,
                                                           (valid && info) ? info + b : nullptr,
                                                           nullptr);
        } else {
            const int g = lane / 32;
            const bool valid = g < cnt;
            const int b = sorted[first + (valid ? g : 0)];
            const int64_t o = offs[b];
            wpm_matrix<V, 32, OP_INV, METHOD, MIXED>(
                a + o, x + o, n, valid, n, n, ns_steps, fill, (valid && info) ? info + b : nullptr,
                nullptr, smem_raw + (size_t)g * wpm_smem_per_matrix<V, 32, MIXED>(), lane % 32);
        }
        __syncthreads();
    }
}

// Orders big_from..64 (big_from = 33 by default, 17 or 25 when the tuner
// finds it faster): one matrix per 256-lane block, four lanes per column.
constexpr int VL_BIG_TPC = 4;

template <class V, int METHOD, int MIXED>
__global__ void __launch_bounds__(64 * VL_BIG_TPC)
k_varlen_big(const V* __restrict__ a, V* x, const int64_t* __restrict__ offs,
             const int32_t* __restrict__ sorted, VarlenPlan* plan, int ns_steps, int fill,
             int32_t* __restrict__ info)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ int s_tile;
    const int j = threadIdx.x / VL_BIG_TPC, h = threadIdx.x % VL_BIG_TPC;
    for (;;) {
        if (threadIdx.x == 0) s_tile = atomicAdd(&plan->next_big, 1);
        __syncthreads();
        const int t = s_tile;
        __syncthreads();
        if (t >= plan->nbig) break;
        int n = 64;
        while (n > plan->big_from && t >= plan->tile_end[n]) --n;
        const int b = sorted[plan->item_start[n] + (t - plan->tile_start[n])];
        const int64_t o = offs[b];
        wpm_matrix<V, 64, OP_INV, METHOD, MIXED, VL_BIG_TPC>(a + o, x + o, n, true, n, n, ns_steps,
                                                             fill, info ? info + b : nullptr,
                                                             nullptr, smem_raw, j, h);
        __syncthreads();
    }
}

// The last bucket for real float matrices by Cholesky without refinement:
// one matrix per four-wave workgroup, padded to order 64 with the identity;
// R and Y = R^{-1} by the sub-blocked routine of leaf_impl.hpp (the updates
// on the matrix cores, five barriers per 16 columns instead of three per
// row), then X = Y Y^T (the Section III.B product, whose leading operation
// count equals Section IV's once R^{-1} skips its zero blocks) as upper 16 x 16
// MFMA tiles, staged in LDS over R for row-major stores.
constexpr int VL_LEAF_NB = 64;
template <int MIXED>
constexpr size_t vl_leaf_smem()
{
    return (size_t)2 * VL_LEAF_NB * lf_ld<float, VL_LEAF_NB>() * sizeof(float) +
           VL_LEAF_NB * sizeof(double);
}

template <int MIXED>
__global__ void __launch_bounds__(LF_THREADS)
k_varlen_leaf(const float* __restrict__ a, float* x, const int64_t* __restrict__ offs,
              const int32_t* __restrict__ sorted, VarlenPlan* plan, int fill,
              int32_t* __restrict__ info)
{
    constexpr int NB = VL_LEAF_NB, LD = lf_ld<float, NB>();
    constexpr int NT = (NB / 16) * (NB / 16 + 1) / 2;       // upper 16 x 16 tiles of X
    constexpr int TPW = (NT + 3) / 4;                        // tiles per wave
    using Acc = typename mfma_acc<float>::type;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    float* Rm = reinterpret_cast<float*>(smem_raw);          // R, then X (row major, upper)
    float* Ym = Rm + NB * LD;                                // R^{-1}
    double* dl = reinterpret_cast<double*>(Ym + NB * LD);    // FP64 pivot accumulators
    __shared__ int s_tile, s_fail;
    const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64;
    const int g = lane / 16, cc = lane % 16;
    for (;;) {
        if (tid == 0) s_tile = atomicAdd(&plan->next_big, 1);
        __syncthreads();
        const int t = s_tile;
        __syncthreads();
        if (t >= plan->nbig) break;
        int n = 64;
        while (n > plan->big_from && t >= plan->tile_end[n]) --n;
        const int b = sorted[plan->item_start[n] + (t - plan->tile_start[n])];
        const float* ab = a + offs[b];
        float* xb = x + offs[b];
        // upper triangle of A (identity beyond n); Y starts at zero
        {
            constexpr int PER = NB * NB / LF_THREADS;
            float v[PER];
#pragma unroll
            for (int u = 0; u < PER; ++u) {
                const int e = tid + LF_THREADS * u, k = e / NB, j = e % NB;
                v[u] = (k == j) ? 1.f : 0.f;
                if (j < n && k < n && k <= j) v[u] = ab[k * n + j];
            }
#pragma unroll
            for (int u = 0; u < PER; ++u) {
                const int e = tid + LF_THREADS * u, k = e / NB, j = e % NB;
                Rm[k * LD + j] = (k <= j) ? v[u] : 0.f;
                Ym[k * LD + j] = 0.f;
            }
        }
        if (MIXED)
            for (int j = tid; j < NB; j += LF_THREADS) dl[j] = (j < n) ? (double)ab[j * n + j] : 1.0;
        __syncthreads();
        const int f = lf_factor_inverse<float, NB, MIXED>(Rm, Ym, dl, n);
        if (tid == 0) s_fail = f;
        // X = Y Y^T: x_ij = sum_{k >= j} y_ik y_jk (i <= j), tile (tr, tc) from k = 16 tc
        Acc xa[TPW];
#pragma unroll
        for (int u = 0; u < TPW; ++u) {
            xa[u] = Acc{0, 0, 0, 0};
            const int q = wave + 4 * u;
            if (q < NT) {
                int tr = 0, rem = q;
                while (rem >= NB / 16 - tr) { rem -= NB / 16 - tr; ++tr; }
                const int tc = tr + rem;
                lf_tile<float>(xa[u], NB - 16 * tc, g, cc,
                               [&](int r, int k) { return Ym[(16 * tr + r) * LD + 16 * tc + k]; },
                               [&](int k, int c) { return Ym[(16 * tc + c) * LD + 16 * tc + k]; });
            }
        }
        __syncthreads();                                     // R is no longer read
#pragma unroll
        for (int u = 0; u < TPW; ++u) {
            const int q = wave + 4 * u;
            if (q < NT) {
                int tr = 0, rem = q;
                while (rem >= NB / 16 - tr) { rem -= NB / 16 - tr; ++tr; }
                const int tc = tr + rem;
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    Rm[(16 * tr + mfma_acc<float>::row(g, v)) * LD + 16 * tc + cc] = xa[u][v];
            }
        }
        __syncthreads();
        const int fl = s_fail;
        for (int e = tid; e < n * n; e += LF_THREADS) {
            const int i = e / n, j = e % n;
            if (j >= i || fill) {
                const float v = (j >= i) ? Rm[i * LD + j] : Rm[j * LD + i];
                xb[e] = fl ? __builtin_nanf("") : v;
            }
        }
        if (tid == 0 && info) info[b] = fl;
        __syncthreads();                                     // LDS free for the next matrix
    }
}

constexpr size_t varlen_plan_bytes() { return (sizeof(VarlenPlan) + 255) / 256 * 256; }

template <class V, int METHOD, int MIXED>
static hipError_t varlen_run(int64_t batch, const int32_t* n_dev, const int64_t* off_dev, int n_max,
                             const void* a, void* x, int ns_steps, int fill, int32_t* info,
                             void* work, hipStream_t s, int big_from)
{
    if (big_from != 17 && big_from != 25) big_from = 33;
    VarlenPlan* plan = reinterpret_cast<VarlenPlan*>(work);
    int32_t* sorted = reinterpret_cast<int32_t*>((char*)work + varlen_plan_bytes());
    const unsigned gb = (unsigned)((batch + 255) / 256);
    hipLaunchKernelGGL(k_vl_init, dim3(1), dim3(256), 0, s, plan);
    hipLaunchKernelGGL(k_vl_count, dim3(gb), dim3(256), 0, s, n_dev, batch, n_max, plan, info);
    hipLaunchKernelGGL(k_vl_scan, dim3(1), dim3(64), 0, s, plan, big_from);
    hipLaunchKernelGGL(k_vl_scatter, dim3(gb), dim3(256), 0, s, n_dev, batch, n_max, plan, sorted);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;

    auto kbig = k_varlen_big<V, METHOD, MIXED>;
    auto kern = k_varlen<V, METHOD, MIXED>;
    constexpr size_t s64 = wpm_smem_per_matrix<V, 64, MIXED>();
    constexpr size_t s32 = 2 * wpm_smem_per_matrix<V, 32, MIXED>();
    static bool attr = false;
    if (!attr) {
        e = hipFuncSetAttribute((const void*)kbig, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)s64);
        if (e != hipSuccess) return e;
        e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)s32);
        if (e != hipSuccess) return e;
        attr = true;
    }
    auto grid_of = [](const void* k, int threads, size_t smem) {
        int per_cu = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, threads, smem) !=
                hipSuccess || per_cu < 1)
            per_cu = 1;
        return (int64_t)device_cus() * per_cu;
    };
    if (n_max >= big_from) {
        bool leaf = false;       // real float, Cholesky, no refinement: the MFMA route
        if constexpr (std::is_same<V, float>::value && METHOD == 0) {
            leaf = !MIXED || ns_steps == 0;
            if (leaf) {
                auto kl = k_varlen_leaf<MIXED>;
                constexpr size_t sl = vl_leaf_smem<MIXED>();
                static bool lattr = false;
                if (!lattr) {
                    e = hipFuncSetAttribute((const void*)kl,
                                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)sl);
                    if (e != hipSuccess) return e;
                    lattr = true;
                }
                hipLaunchKernelGGL(kl, dim3((unsigned)grid_of((const void*)kl, LF_THREADS, sl)),
                                   dim3(LF_THREADS), sl, s, (const float*)a, (float*)x, off_dev,
                                   sorted, plan, fill, info);
            }
        }
        if (!leaf)
            hipLaunchKernelGGL(kbig,
                               dim3((unsigned)grid_of((const void*)kbig, 64 * VL_BIG_TPC, s64)),
                               dim3(64 * VL_BIG_TPC), s64, s, (const V*)a, (V*)x, off_dev, sorted,
                               plan, ns_steps, fill, info);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    const size_t smem = n_max > 16 ? s32 : 0;
    hipLaunchKernelGGL(kern, dim3((unsigned)grid_of((const void*)kern, 64, smem)), dim3(64), smem, s,
                       (const V*)a, (V*)x, off_dev, sorted, plan, ns_steps, fill, info);
    return hipGetLastError();
}

template <class V>
static hipError_t varlen_dispatch(int64_t batch, const int32_t* n_dev, const int64_t* off_dev,
                                  int n_max, const void* a, void* x, int method, int mixed,
                                  int ns_steps, int fill, int32_t* info, void* work, hipStream_t s,
                                  int big_from)
{
    constexpr bool f32 = sizeof(typename vt<V>::real) == 4;
    if (mixed) {
        if constexpr (f32) {
            if (method == 0)
                return varlen_run<V, 0, 1>(batch, n_dev, off_dev, n_max, a, x, ns_steps, fill, info,
                                           work, s, big_from);
            return varlen_run<V, 1, 1>(batch, n_dev, off_dev, n_max, a, x, ns_steps, fill, info,
                                       work, s, big_from);
        }
        return hipErrorNotSupported;
    }
    if (method == 0)
        return varlen_run<V, 0, 0>(batch, n_dev, off_dev, n_max, a, x, 0, fill, info, work, s,
                                   big_from);
    return varlen_run<V, 1, 0>(batch, n_dev, off_dev, n_max, a, x, 0, fill, info, work, s,
                               big_from);
}

}  // namespace ci
