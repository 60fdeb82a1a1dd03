// Batched resampling: many independent instances of uneven size (a particle
// MCMC run or a serving batch runs many filters at once; Sec. 1 of the paper
// motivates the Metropolis resampler by exactly this repeated use) in one
// graph replay of three persistent launches.
//
//   launch 1  tile reductions of every stratified/systematic (and adaptive
//             Metropolis) instance
//   launch 2  the per-instance tables (one block each; an adaptive
//             Metropolis table computes eq. (5)'s B)
//   launch 3  Metropolis chains and stratified/systematic fills of every
//             instance, each item followed by the ancestor-indexed copy of
//             its rows (fused: the ancestors are still in LDS)
//
// Each launch is a persistent grid walking a static work list (items sorted
// by decreasing cost, dealt out round-robin), so the grid never depends on
// the data. Phases are ordered by kernel boundaries rather than by blocks
// waiting on device-scope flags: on MI355X every cross-XCD publication needs
// an L2 write-back, which costs far more than a launch boundary inside a
// graph. Every item runs the same device bodies as the single-instance entry
// points, so each instance's ancestors are bit-identical alone and in any
// batch.
#include <hip/hip_runtime.h>

#include "common.h"
#include "launch.h"
#include "metropolis_impl.h"
#include "prefix.h"
#include "prefix_impl.h"

namespace rs {
namespace {

using namespace pfx;

constexpr int kThreads = kTileThreads;  // every batched launch uses 256-thread blocks
constexpr int64_t kTableLdsTiles = 4096;

__global__ __launch_bounds__(kThreads) void batch_tile_kernel(const BatchInstance *insts,
                                                              const int2 *items, int32_t n_items)
{
    for (int32_t it = blockIdx.x; it < n_items; it += gridDim.x) {
        __syncthreads();  // LDS of the previous item is free
        const int2 item = items[it];
        const BatchInstance &I = insts[item.x];
        tile_reduce_body(I.lw, I.P, item.y, I.ws);
    }
}

__global__ __launch_bounds__(kThreads) void batch_table_kernel(const BatchInstance *insts,
                                                               const int32_t *items,
                                                               int32_t n_items, int use_lds,
                                                               uint32_t instance_add)
{
    extern __shared__ double sh_tab[];
    for (int32_t it = blockIdx.x; it < n_items; it += gridDim.x) {
        __syncthreads();
        const BatchInstance &I = insts[items[it]];
        const WsView ws = ws_view(I.ws, I.P);
        const int64_t n = num_tiles(I.P);
        const bool lds = use_lds != 0;  // LDS sized for the largest table of the batch
        double *bound = lds ? sh_tab : ws.bound;
        int32_t *count = lds ? reinterpret_cast<int32_t *>(sh_tab + n) : ws.count;
        const uint32_t inst = I.instance + instance_add;
        if (I.kind == kStratified)
            table_body<kStratified>(I.P, I.seed, inst, I.ws, I.status, nullptr, bound, count);
        else if (I.kind == kSystematic)
            table_body<kSystematic>(I.P, I.seed, inst, I.ws, I.status, nullptr, bound, count);
        else  // adaptive Metropolis: eq. (5)'s B (capped by I.B) into the header
            table_body<kAdaptiveB>(I.P, I.seed, inst, I.ws, I.status, nullptr, bound, count,
                                   I.eps, I.B, nullptr);
    }
}

// A Metropolis item: chains [first, first + count) of one instance, then the
// copy of their rows. sh_anc holds the item's ancestors for the copy; w is
// LDS-staged weights or the instance's lw.
template <int UNROLL>
__device__ void metropolis_item(const BatchInstance &I, uint32_t B, uint32_t inst, int64_t first,
                                int64_t count, float *staged, int32_t *sh_anc)
{
    const uint32_t P = (uint32_t)I.P;
    const float *w = I.lw;
    if (staged) {
        for (uint32_t i = threadIdx.x; i < P; i += kThreads) staged[i] = I.lw[i];
        __syncthreads();
        w = staged;
    }
    int fl = 0;
    for (int64_t r = threadIdx.x; r < count; r += kThreads) {
        const uint32_t i = (uint32_t)(first + r);
        fl |= mh::weight_flags(w[i]);
        const int32_t a = (int32_t)mh::chain<UNROLL>(w, P, B, I.seed, inst, i);
        I.anc[i] = a;
        if (I.x_in) sh_anc[r] = a;
    }
    raise_flags(I.status, fl);
    if (I.x_in) {
        __syncthreads();
        int cf = 0;
        copy_rows_from_lds(sh_anc, first, first, first + count, I.x_in, I.x_out, I.D, I.P, &cf);
        raise_flags(I.status, cf);
    }
}

template <int UNROLL>
__global__ __launch_bounds__(kThreads) void batch_main_kernel(const BatchInstance *insts,
                                                              const int2 *items, int32_t n_items,
                                                              int32_t chains_per_item,
                                                              int64_t lds_max_p,
                                                              uint32_t instance_add)
{
    extern __shared__ double sh_main[];  // [kChunk ints | union(kTile doubles, staged lw)]
    int32_t *sh_anc = reinterpret_cast<int32_t *>(sh_main);
    double *Cs = sh_main + kChunk / 2;
    float *staging = reinterpret_cast<float *>(Cs);
    for (int32_t it = blockIdx.x; it < n_items; it += gridDim.x) {
        __syncthreads();
        const int2 item = items[it];
        const BatchInstance &I = insts[item.x];
        const uint32_t inst = I.instance + instance_add;
        if (I.kind == kMetropolisKind || I.kind == kAdaptiveKind) {
            const int64_t first = (int64_t)item.y * chains_per_item;
            const int64_t count = min((int64_t)chains_per_item, I.P - first);
            // an adaptive instance reads the B its table left in the header
            const uint32_t B = I.kind == kAdaptiveKind ? ws_view(I.ws, I.P).h->B : I.B;
            metropolis_item<UNROLL>(I, B, inst, first, count,
                                    I.P <= lds_max_p ? staging : nullptr, sh_anc);
        } else if (I.kind == kStratified) {
            fill_body<kStratified, false>(I.lw, I.anc, I.off, I.P, I.seed, inst, nullptr, I.ws,
                                          item.y, I.x_in, I.x_out, I.D, I.status, Cs, sh_anc,
                                          nullptr);
        } else {
            fill_body<kSystematic, false>(I.lw, I.anc, I.off, I.P, I.seed, inst, nullptr, I.ws,
                                          item.y, I.x_in, I.x_out, I.D, I.status, Cs, sh_anc,
                                          nullptr);
        }
    }
}

uint32_t grid_of(int32_t items, int32_t blocks) { return (uint32_t)max(1, min(items, blocks)); }

// acc[k] += log of instance k's mean weight, lse_k - log P_k (the likelihood
// factor of Sec. 1's weighting step), from the header its table left; NaN
// for instances without a table (fixed-B Metropolis, P = 0).
__global__ __launch_bounds__(kThreads) void batch_log_mean_weight_kernel(const BatchInstance *insts,
                                                                         int32_t n, double *acc)
{
    for (int32_t k = blockIdx.x * kThreads + threadIdx.x; k < n; k += gridDim.x * kThreads) {
        const BatchInstance &I = insts[k];
        const bool table = I.ws && I.P > 0 && I.kind != kMetropolisKind;
        acc[k] += table ? ws_view(I.ws, I.P).h->lse - log((double)I.P) : (double)NAN;
    }
}

// out[k] = the Metropolis iterations instance k ran in the plan's last run:
// eq. (5)'s count from its table for an adaptive instance, its B for a
// fixed one, 0 for other kinds and empty instances.
__global__ __launch_bounds__(kThreads) void batch_iterations_kernel(const BatchInstance *insts,
                                                                    int32_t n, uint32_t *out)
{
    for (int32_t k = blockIdx.x * kThreads + threadIdx.x; k < n; k += gridDim.x * kThreads) {
        const BatchInstance &I = insts[k];
        uint32_t B = 0;
        if (I.P > 0 && I.kind == kMetropolisKind) B = I.B;
        if (I.P > 0 && I.kind == kAdaptiveKind && I.ws) B = ws_view(I.ws, I.P).h->B;
        out[k] = B;
    }
}

}  // namespace

int launch_batch_iterations(const BatchInstance *insts, int32_t n, uint32_t *out,
                            hipStream_t stream)
{
    const uint32_t grid = (uint32_t)max(1, min((n + kThreads - 1) / kThreads, 1024));
    hipLaunchKernelGGL(batch_iterations_kernel, dim3(grid), dim3(kThreads), 0, stream, insts, n,
                       out);
    return launch_status();
}

int launch_batch(const BatchLaunch &L, hipStream_t stream)
{
    if (L.n_tile_items > 0)
        hipLaunchKernelGGL(batch_tile_kernel, dim3(grid_of(L.n_tile_items, L.blocks)),
                           dim3(kThreads), 0, stream, L.insts, L.tile_items, L.n_tile_items);
    if (L.n_table_items > 0) {
        const int64_t n = L.max_table_tiles;
        const int use_lds = n <= kTableLdsTiles ? 1 : 0;
        const size_t smem = use_lds ? (size_t)n * (sizeof(double) + sizeof(int32_t)) : 0;
        hipLaunchKernelGGL(batch_table_kernel, dim3(grid_of(L.n_table_items, L.blocks)),
                           dim3(kThreads), smem, stream, L.insts, L.table_items, L.n_table_items,
                           use_lds, L.instance_add);
    }
    if (L.n_main_items > 0) {
        const size_t smem = L.smem_main;
        const dim3 grid(grid_of(L.n_main_items, L.blocks)), block(kThreads);
#define RS_BATCH_CASE(U)                                                                         \
    case U: {                                                                                    \
        if (allow_dynamic_lds(reinterpret_cast<const void *>(&batch_main_kernel<U>), smem))     \
            return -3;                                                                           \
        hipLaunchKernelGGL(batch_main_kernel<U>, grid, block, smem, stream, L.insts, L.main_items, \
                           L.n_main_items, L.chains_per_item, L.lds_max_p, L.instance_add);      \
        break;                                                                                   \
    }
        switch (L.unroll) {
            RS_BATCH_CASE(2)
            RS_BATCH_CASE(4)
            RS_BATCH_CASE(8)
            RS_BATCH_CASE(16)
        default:
            return -1;
        }
#undef RS_BATCH_CASE
    }
    return launch_status();
}

int launch_batch_log_mean_weight(const BatchInstance *insts, int32_t n, double *acc,
                                 hipStream_t stream)
{
    const uint32_t grid = (uint32_t)max(1, min((n + kThreads - 1) / kThreads, 1024));
    hipLaunchKernelGGL(batch_log_mean_weight_kernel, dim3(grid), dim3(kThreads), 0, stream, insts,
                       n, acc);
    return launch_status();
}

}  // namespace rs
