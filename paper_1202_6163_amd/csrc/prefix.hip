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
//  2. table_kernel (one block) rescales the tile sums to the
//     global max, scans them into tile boundaries B_t, counts for every
//     boundary the draw points below it (stratified/systematic draws are
//     non-decreasing, so this is a short search near B_t / (W/P)), and lays
//     out the fill blocks: one per tile, plus one per further 2048 draws of a
//     tile that owns more.
//  3. fill_kernel: each block re-reads its tile of lw, rebuilds the tile's
//     cumulative weights in LDS with a wave-level scan, and locates each of
//     its draw points there, writing ancestors in order.
// HBM traffic is two reads of lw and one write of anc; the cumulative weights
// are stored only on request. The multinomial draws are unsorted, so that
// resampler stores C (launch 3m) and bisects it per draw (launch 4m).
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

template <int KIND>
__global__ __launch_bounds__(kTileThreads) void fill_kernel(const float *__restrict__ lw,
                                                            int32_t *__restrict__ anc, int64_t P,
                                                            uint64_t seed, uint32_t instance,
                                                            double *cumw, char *ws_raw)
{
    __shared__ double Cs[kTile];
    fill_body<KIND>(lw, anc, P, seed, instance, cumw, ws_raw, blockIdx.x, nullptr, nullptr, 0,
                    nullptr, Cs, nullptr);
}

// ------------------------------------------------------ multinomial
// Launch 3m: one block per tile writes C' for the tile.
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
}

// Launch 4m: each thread draws two points (one Philox block) and locates
// each by bisection over the tile boundaries (staged in LDS when they fit),
// then over the tile's cumulative weights.
__global__ __launch_bounds__(256) void multinomial_search_kernel(const double *__restrict__ C,
                                                                 int32_t *__restrict__ anc,
                                                                 int64_t P, uint64_t seed,
                                                                 uint32_t instance, char *ws_raw,
                                                                 int lds_bounds)
{
    extern __shared__ double sh_bound[];
    const WsView ws = ws_view(ws_raw, P);
    const int64_t n = num_tiles(P);
    const int flags = ws.h->flags;
    const double *bound = ws.bound;
    if (lds_bounds) {
        for (int64_t t = threadIdx.x; t < n; t += blockDim.x) sh_bound[t] = ws.bound[t];
        __syncthreads();
        bound = sh_bound;
    }
    const double W = ws.h->W;
    const int64_t pairs = (P + 1) >> 1;
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < pairs;
         p += (int64_t)gridDim.x * blockDim.x) {
        if (flags) {
            anc[2 * p] = (int32_t)(2 * p);
            if (2 * p + 1 < P) anc[2 * p + 1] = (int32_t)(2 * p + 1);
            continue;
        }
        const Block4 b = philox(seed, (uint32_t)p, instance, 0u, kTagMultinomial);
        const double xs[2] = {unit53(b.r0, b.r1) * W, unit53(b.r2, b.r3) * W};
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int64_t i = 2 * p + h;
            if (i >= P) break;
            const double xw = fmin(xs[h], below(W));
            int64_t lo = 0, hi = n - 1;  // first tile with bound > xw
            while (lo < hi) {
                const int64_t mid = (lo + hi) >> 1;
                if (bound[mid] > xw) hi = mid;
                else lo = mid + 1;
            }
            const int64_t t = lo;
            const double xt = fmin(xs[h], below(bound[t]));
            const int64_t base = t * kTile;
            int64_t a = 0, z = min((int64_t)kTile, P - base) - 1;  // first j with C > xt
            while (a < z) {
                const int64_t mid = (a + z) >> 1;
                if (C[base + mid] > xt) z = mid;
                else a = mid + 1;
            }
            anc[i] = (int32_t)(base + a);
        }
    }
}

}  // namespace

// ---------------------------------------------------------------- launchers
int launch_prefix(int kind, const float *lw, int32_t *anc, int64_t P, uint64_t seed,
                  uint32_t instance, double *cumw, void *ws, int32_t *status,
                  hipStream_t stream)
{
    const int64_t n = num_tiles(P);
    char *w = static_cast<char *>(ws);
    const dim3 tb(kTileThreads);
    const dim3 fill_grid((uint32_t)(n + max_overflow_chunks(P)));
    hipLaunchKernelGGL(tile_reduce_kernel, dim3((uint32_t)n), tb, 0, stream, lw, P, w);
    switch (kind) {
    case kStratified:
        launch_table<kStratified>(P, seed, instance, w, status, nullptr, stream);
        hipLaunchKernelGGL(fill_kernel<kStratified>, fill_grid, tb, 0, stream, lw, anc, P, seed,
                           instance, cumw, w);
        break;
    case kSystematic:
        launch_table<kSystematic>(P, seed, instance, w, status, nullptr, stream);
        hipLaunchKernelGGL(fill_kernel<kSystematic>, fill_grid, tb, 0, stream, lw, anc, P, seed,
                           instance, cumw, w);
        break;
    case kMultinomial: {
        double *C = cumw ? cumw : reinterpret_cast<double *>(w + ws_layout(P, true).cumw);
        launch_table<kMultinomial>(P, seed, instance, w, status, nullptr, stream);
        hipLaunchKernelGGL(cumulative_kernel, dim3((uint32_t)n), tb, 0, stream, lw, P, C, w);
        const int lds_bounds = n <= 4096 ? 1 : 0;
        const size_t smem = lds_bounds ? (size_t)n * sizeof(double) : 0;
        const int64_t pairs = (P + 1) >> 1;
        int64_t grid = (pairs + 255) / 256;
        if (grid > 8192) grid = 8192;
        hipLaunchKernelGGL(multinomial_search_kernel, dim3((uint32_t)grid), dim3(256), smem, stream,
                           C, anc, P, seed, instance, w, lds_bounds);
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
