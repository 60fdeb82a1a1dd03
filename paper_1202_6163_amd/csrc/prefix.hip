// Prefix-sum resamplers on gfx950: stratified, systematic, multinomial, and
// the log-sum-exp reduction they share.
//
// Method (Sec. 2 of the paper): the multinomial, stratified and systematic
// resamplers need the collective prefix sum C_j = sum_{k<=j} w_k of the
// weights w_k = exp(lw_k - max lw), then pick for draw point x the ancestor
// a(x) = min{j : C_j > x} (for x >= W = C_{P-1}: the first j with C_j = W).
//   stratified:  x_i = (i + U_i) W / P      (one uniform per stratum)
//   systematic:  x_i = (i + U) W / P        (one shared uniform)
//   multinomial: x_i = U_i W                (independent uniforms)
//
// Design on MI355X.
//  1. tile_reduce_kernel streams lw once: per 1024-weight tile the max, the
//     sum of exp(lw - tile max) in binary64 and the data flags.
//  2. fill_kernel: every block rescales the tile sums to the global max and
//     scans them into the tile boundaries B_t in LDS (a few KB: the same
//     computation in every block costs less than another dependent launch),
//     counts the draws below its tile's two boundaries (stratified/systematic
//     draws are non-decreasing, so this is a short search near B / (W/P)),
//     re-reads its tile of lw, rebuilds the tile's cumulative weights in LDS
//     with a wave-level scan and locates each of its draws there, writing
//     ancestors in order. Blocks beyond one per tile take the draws of heavy
//     tiles by 2048-wide windows of draw index. Above 64 tiles a one-block
//     table launch computes boundaries and counts once instead.
//     With an offspring array each tile block also writes o_j for its tile's
//     particles, counted from the sorted ancestors it holds in LDS.
// HBM traffic is two reads of lw and one write of anc (and/or off); the
// cumulative weights are stored only on request. The multinomial draws are
// unsorted, so that resampler stores C (launch 3m) and searches it per draw
// (launch 4m): every 64th C' staged in LDS, then the 64 C' of the draw's
// group in HBM.
//
// Rounding: inside a tile C'_j = min(B_{t-1} + L_j, B_t), where L_j is a
// zero-weight-aware running maximum of the tile's scan, and C'_j = B_t from
// the tile's last positive weight on. This keeps C' non-decreasing across
// tiles although the tile sums and the in-tile scans round differently, and
// keeps zero-weight particles unselectable. C' agrees with the binary64
// left-to-right sum to a few ulps.
#include <hip/hip_runtime.h>

#include "common.h"
#include "launch.h"
#include "prefix.h"
#include "prefix_impl.h"

namespace rs {
namespace {

using namespace pfx;

// Tables keep their per-tile arrays in LDS up to this many tiles.
constexpr int64_t kTableLdsTiles = 4096;

__global__ __launch_bounds__(kTileThreads) void tile_reduce_kernel(const float *__restrict__ lw,
                                                                   int64_t P, char *ws_raw)
{
    tile_reduce_body(lw, P, blockIdx.x, ws_raw);
}

template <int KIND, bool LDS>
__global__ __launch_bounds__(kTileThreads) void table_kernel(int64_t P, uint64_t seed,
                                                             uint32_t instance, char *ws_raw,
                                                             int32_t *status, double *lse_out,
                                                             double eps, uint32_t B_max,
                                                             uint32_t *B_used)
{
    extern __shared__ double sh_tab[];  // [n] boundaries, then [n] counts
    const WsView ws = ws_view(ws_raw, P);
    const int64_t n = num_tiles(P);
    double *bound = LDS ? sh_tab : ws.bound;
    int32_t *count = LDS ? reinterpret_cast<int32_t *>(sh_tab + n) : ws.count;
    table_body<KIND>(P, seed, instance, ws_raw, status, lse_out, bound, count, eps, B_max, B_used);
}

template <int KIND>
void launch_table(int64_t P, uint64_t seed, uint32_t instance, char *w, int32_t *status,
                  double *lse_out, hipStream_t stream, double eps = 0.0, uint32_t B_max = 0,
                  uint32_t *B_used = nullptr)
{
    const int64_t n = num_tiles(P);
    if (n <= kTableLdsTiles) {
        const size_t smem = (size_t)n * (sizeof(double) + sizeof(int32_t));
        hipLaunchKernelGGL((table_kernel<KIND, true>), dim3(1), dim3(kTileThreads), smem, stream,
                           P, seed, instance, w, status, lse_out, eps, B_max, B_used);
    } else {
        hipLaunchKernelGGL((table_kernel<KIND, false>), dim3(1), dim3(kTileThreads), 0, stream, P,
                           seed, instance, w, status, lse_out, eps, B_max, B_used);
    }
}

template <int KIND, bool FUSED>
__global__ __launch_bounds__(kTileThreads) void fill_kernel(const float *__restrict__ lw,
                                                            int32_t *__restrict__ anc,
                                                            int32_t *__restrict__ off, int64_t P,
                                                            uint64_t seed, uint32_t instance,
                                                            double *cumw, char *ws_raw,
                                                            int32_t *status, Rows rows)
{
    __shared__ double Cs[kTile];
    __shared__ int32_t sh_anc[kChunk];  // the block's ancestors (offspring counts, row copy)
    extern __shared__ double sh_bound[];  // FUSED: the n tile boundaries
    fill_body<KIND, FUSED>(lw, anc, off, P, seed, instance, cumw, ws_raw, blockIdx.x, rows.x_in,
                           rows.x_out, rows.D, status, Cs, sh_anc, sh_bound);
}

// Stratified/systematic: with at most kFusedTableTiles tiles the fill blocks
// rebuild the boundaries themselves (two launches); beyond that a table
// launch computes them once (three launches). Same values either way: both
// run pfx::boundaries and pfx::count_below.
template <int KIND>
void launch_fill(const float *lw, int32_t *anc, int32_t *off, int64_t P, uint64_t seed,
                 uint32_t instance, double *cumw, char *w, int32_t *status, hipStream_t stream,
                 const Rows &rows)
{
    const int64_t n = num_tiles(P);
    const dim3 grid((uint32_t)num_fill_blocks(P)), tb(kTileThreads);
    if (n <= kFusedTableTiles) {
        hipLaunchKernelGGL((fill_kernel<KIND, true>), grid, tb, (size_t)n * sizeof(double), stream,
                           lw, anc, off, P, seed, instance, cumw, w, status, rows);
    } else {
        launch_table<KIND>(P, seed, instance, w, status, nullptr, stream);
        hipLaunchKernelGGL((fill_kernel<KIND, false>), grid, tb, 0, stream, lw, anc, off, P, seed,
                           instance, cumw, w, status, rows);
    }
}

// ------------------------------------------------------ multinomial
// Launch 3m: one block per tile writes C' for the tile, and the last C' of
// every kSubStride-wide group into the compact array ws.sub (the group that
// holds P - 1 takes the C' at its padded end, which equals W like C'_{P-1}).
__global__ __launch_bounds__(kTileThreads) void cumulative_kernel(const float *__restrict__ lw,
                                                                  int64_t P, double *C,
                                                                  char *ws_raw)
{
    __shared__ double Cs[kTile];
    const WsView ws = ws_view(ws_raw, P);
    const int64_t t = blockIdx.x;
    float v[4];
    load_tile4(lw, P, t, v);
    if (ws.h->flags) {
        const int64_t base = t * kTile + 4 * (int64_t)threadIdx.x;
        for (int k = 0; k < 4; ++k)
            if (base + k < P) C[base + k] = (double)NAN;
        return;
    }
    const double Blo = t > 0 ? ws.bound[t - 1] : 0.0;
    double Cv[4];
    tile_cumulative(v, ws.h->m, Blo, ws.bound[t], Cs, Cv);
    store_cumw(C, P, t, Cv);
    const int64_t S = sub_stride(P), ns = num_sub(P);
    const int64_t e = t * kTile + 4 * (int64_t)threadIdx.x + 3;  // this thread's last element
    if ((e + 1) % S == 0 && e / S < ns)
        ws.sub[e / S] = Cv[3];
    else if (S > kTile && t == num_tiles(P) - 1 && threadIdx.x == kTileThreads - 1)
        ws.sub[ns - 1] = Cv[3];  // last group ends past the last tile
}

// First index in [0, len) with a[i] > x, given a[len - 1] > x: branchless
// bisection, ceil(log2 len) steps whatever x is.
__device__ __forceinline__ int64_t first_above(const double *a, int64_t len, double x)
{
    int64_t base = 0;
    while (len > 1) {
        const int64_t half = len >> 1;
        if (a[base + half - 1] <= x) base += half;
        len -= half;
    }
    return base;
}

// Launch 4m: a persistent grid of 1024-thread blocks. Each block stages
// ws.sub (the last C' of every group of S = sub_stride(P) particles; at most
// 128 KB) in LDS; each thread draws kDraws points (two per Philox block) and
// locates them side by side (their memory round trips overlap): bisection
// over the staged group ends, then over the group's S cumulative weights in
// global memory (S = 64 up to 2^20 particles: six dependent reads within four
// cache lines).
constexpr int kDraws = 4;
constexpr int kSearchThreads = 1024;

__global__ __launch_bounds__(kSearchThreads) void multinomial_search_kernel(
    const double *__restrict__ C, int32_t *__restrict__ anc, int64_t P, uint64_t seed,
    uint32_t instance, char *ws_raw, Rows rows)
{
    extern __shared__ double sh_sub[];
    const WsView ws = ws_view(ws_raw, P);
    const int64_t S = sub_stride(P), ns = num_sub(P);
    const int flags = ws.h->flags;
    const double W = ws.h->W;
    if (!flags) {
        for (int64_t k = threadIdx.x; k < ns; k += kSearchThreads) sh_sub[k] = ws.sub[k];
        __syncthreads();
    }
    const double capW = below(W);
    const int64_t groups = (P + kDraws - 1) / kDraws;
    for (int64_t q = blockIdx.x * (int64_t)kSearchThreads + threadIdx.x; q < groups;
         q += (int64_t)gridDim.x * kSearchThreads) {
        const int64_t i0 = q * kDraws;
        if (flags) {
            for (int k = 0; k < kDraws; ++k) {
                if (i0 + k < P) {
                    anc[i0 + k] = (int32_t)(i0 + k);
                    if (rows.x_in) copy_row(rows, i0 + k, i0 + k, 0, 1);
                }
            }
            continue;
        }
        double x[kDraws];
#pragma unroll
        for (int p = 0; p < kDraws / 2; ++p) {
            const Block4 b = philox(seed, (uint32_t)(i0 / 2 + p), instance, 0u, kTagMultinomial);
            x[2 * p] = fmin(unit53(b.r0, b.r1) * W, capW);
            x[2 * p + 1] = fmin(unit53(b.r2, b.r3) * W, capW);
        }
        int64_t gk[kDraws];
#pragma unroll
        for (int k = 0; k < kDraws; ++k) gk[k] = first_above(sh_sub, ns, x[k]);
        int64_t j[kDraws];
#pragma unroll
        for (int k = 0; k < kDraws; ++k) {
            const int64_t base = gk[k] * S;
            j[k] = base + first_above(C + base, min(S, P - base), x[k]);
        }
        if (i0 + kDraws <= P && (((uintptr_t)(anc + i0)) & 15) == 0) {
            *reinterpret_cast<int4 *>(anc + i0) =
                make_int4((int32_t)j[0], (int32_t)j[1], (int32_t)j[2], (int32_t)j[3]);
        } else {
#pragma unroll
            for (int k = 0; k < kDraws; ++k)
                if (i0 + k < P) anc[i0 + k] = (int32_t)j[k];
        }
        if (rows.x_in) {
#pragma unroll
            for (int k = 0; k < kDraws; ++k)
                if (i0 + k < P) copy_row(rows, i0 + k, j[k], 0, 1);
        }
    }
}

}  // namespace

// ---------------------------------------------------------------- launchers
int launch_prefix(int kind, const float *lw, int32_t *anc, int32_t *off, int64_t P, uint64_t seed,
                  uint32_t instance, double *cumw, void *ws, int32_t *status,
                  hipStream_t stream, const Rows &rows)
{
    const int64_t n = num_tiles(P);
    char *w = static_cast<char *>(ws);
    const dim3 tb(kTileThreads);
    hipLaunchKernelGGL(tile_reduce_kernel, dim3((uint32_t)n), tb, 0, stream, lw, P, w);
    switch (kind) {
    case kStratified:
        launch_fill<kStratified>(lw, anc, off, P, seed, instance, cumw, w, status, stream, rows);
        break;
    case kSystematic:
        launch_fill<kSystematic>(lw, anc, off, P, seed, instance, cumw, w, status, stream, rows);
        break;
    case kMultinomial: {
        double *C = cumw ? cumw : reinterpret_cast<double *>(w + ws_layout(P, true).cumw);
        launch_table<kMultinomial>(P, seed, instance, w, status, nullptr, stream);
        hipLaunchKernelGGL(cumulative_kernel, dim3((uint32_t)n), tb, 0, stream, lw, P, C, w);
        const size_t smem = (size_t)num_sub(P) * sizeof(double);
        static size_t granted = 0;  // dynamic LDS above the default needs the attribute
        if (smem > granted) {
            if (hipFuncSetAttribute(reinterpret_cast<const void *>(&multinomial_search_kernel),
                                    hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)smem) != hipSuccess)
                return launch_status();
            granted = smem;
        }
        const int64_t per_block = (int64_t)kDraws * kSearchThreads;
        const int64_t need = (P + per_block - 1) / per_block;
        const int64_t grid = need < 1 ? 1 : (need > 2048 ? 2048 : need);
        hipLaunchKernelGGL(multinomial_search_kernel, dim3((uint32_t)grid), dim3(kSearchThreads),
                           smem, stream, C, anc, P, seed, instance, w, rows);
        break;
    }
    default:
        return -1;
    }
    return launch_status();
}

int launch_adaptive_B(const float *lw, int64_t P, double eps, uint32_t B_max, void *ws,
                      uint32_t *B_used, int32_t *status, hipStream_t stream)
{
    char *w = static_cast<char *>(ws);
    hipLaunchKernelGGL(tile_reduce_kernel, dim3((uint32_t)num_tiles(P)), dim3(kTileThreads), 0,
                       stream, lw, P, w);
    launch_table<kAdaptiveB>(P, 0, 0u, w, status, nullptr, stream, eps, B_max, B_used);
    return launch_status();
}

const uint32_t *adaptive_B_slot(const void *ws)
{
    return &static_cast<const WsHeader *>(ws)->B;
}

int launch_log_sum_exp(const float *lw, int64_t P, double *out, void *ws, int32_t *status,
                       hipStream_t stream)
{
    char *w = static_cast<char *>(ws);
    hipLaunchKernelGGL(tile_reduce_kernel, dim3((uint32_t)num_tiles(P)), dim3(kTileThreads), 0,
                       stream, lw, P, w);
    launch_table<kLogSumExp>(P, 0, 0u, w, status, out, stream);
    return launch_status();
}

}  // namespace rs
