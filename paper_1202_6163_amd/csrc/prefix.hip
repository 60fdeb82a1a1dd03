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
//  2. table_kernel (up to 8 blocks): the tile sums rescaled to the global
//     max and scanned into the tile boundaries B_t, the number of draw points
//     below each boundary (stratified/systematic draws are non-decreasing, so
//     this is a short search near B / (W/P)) and the owners of the overflow
//     windows. Up to 64 tiles the fill blocks do this themselves instead.
//  3. fill_kernel: each block re-reads its tile of lw, rebuilds the tile's
//     cumulative weights in LDS with a wave-level scan and locates each of
//     its draws there, writing ancestors in order, and the tile's offspring
//     o_j counted from the sorted ancestors it holds in LDS. Blocks beyond one
//     per tile take the rest of heavy tiles by 2044-wide windows of draw
//     index.
// HBM traffic is two reads of lw and one write of anc (and/or off); the
// cumulative weights are stored only on request. The multinomial draws are
// unsorted, so that resampler stores C (launch 3m) and searches it per draw
// (launch 4m): the particles are split in eight parts, one per XCD, each
// searched by the blocks that XCD runs (every 16th C' of the part staged in
// LDS, then one 128-byte line of C).
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

// Tables keep their boundaries in LDS up to this many tiles (128 KB).
constexpr int64_t kTableLdsTiles = 16384;

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
    extern __shared__ double sh_tab[];  // [n] boundaries, then the block's counts
    const WsView ws = ws_view(ws_raw, P);
    const int64_t n = num_tiles(P);
    double *bound = LDS ? sh_tab : ws.bound;
    int32_t *count = LDS ? reinterpret_cast<int32_t *>(sh_tab + n) : ws.count;
    table_body<KIND>(P, seed, instance, ws_raw, status, lse_out, bound, count, eps, B_max, B_used,
                     blockIdx.x, gridDim.x);
}

// Stratified/systematic tables with LDS boundaries split the counts over up
// to kTableParts blocks; the rest run one block.
constexpr int64_t kTableParts = 8;

template <int KIND>
int launch_table(int64_t P, uint64_t seed, uint32_t instance, char *w, int32_t *status,
                  double *lse_out, hipStream_t stream, double eps = 0.0, uint32_t B_max = 0,
                  uint32_t *B_used = nullptr)
{
    const int64_t n = num_tiles(P);
    if (n <= kTableLdsTiles) {
        int64_t parts = 1;
        if (KIND == kStratified || KIND == kSystematic) {
            parts = (n + kTileThreads - 1) / kTileThreads;
            parts = parts > kTableParts ? kTableParts : parts;
        }
        const int64_t slice = (n + parts - 1) / parts + 2;  // a block's counts (one extra)
        const size_t smem = (size_t)n * sizeof(double) + (size_t)slice * sizeof(int32_t);
        if (allow_dynamic_lds(reinterpret_cast<const void *>(&table_kernel<KIND, true>), smem))
            return -3;
        hipLaunchKernelGGL((table_kernel<KIND, true>), dim3((uint32_t)parts), dim3(kTileThreads),
                           smem, stream, P, seed, instance, w, status, lse_out, eps, B_max,
                           B_used);
    } else {
        hipLaunchKernelGGL((table_kernel<KIND, false>), dim3(1), dim3(kTileThreads), 0, stream, P,
                           seed, instance, w, status, lse_out, eps, B_max, B_used);
    }
    return 0;
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
int launch_fill(const float *lw, int32_t *anc, int32_t *off, int64_t P, uint64_t seed,
                 uint32_t instance, double *cumw, char *w, int32_t *status, hipStream_t stream,
                 const Rows &rows)
{
    const int64_t n = num_tiles(P);
    const dim3 grid((uint32_t)num_fill_blocks(P)), tb(kTileThreads);
    if (n <= kFusedTableTiles) {
        hipLaunchKernelGGL((fill_kernel<KIND, true>), grid, tb, (size_t)n * sizeof(double), stream,
                           lw, anc, off, P, seed, instance, cumw, w, status, rows);
    } else {
        if (const int rc = launch_table<KIND>(P, seed, instance, w, status, nullptr, stream)) return rc;
        hipLaunchKernelGGL((fill_kernel<KIND, false>), grid, tb, 0, stream, lw, anc, off, P, seed,
                           instance, cumw, w, status, rows);
    }
    return 0;
}

// ------------------------------------------------------ multinomial
// Launch 3m: one block per tile writes C' for the tile, and into ws.sub the
// last C' of every sub_stride(P)-particle group of each part (the last group
// of a part ends at the part's end).
__global__ __launch_bounds__(kTileThreads) void cumulative_kernel(const float *__restrict__ lw,
                                                                  int64_t P, double *C,
                                                                  char *ws_raw, uint64_t seed,
                                                                  uint32_t instance)
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
    double w[4], Cv[4];
    tile_weights(v, ws.h->m, w);
    tile_cumulative(w, Blo, ws.bound[t], Cs, Cv);
    store_cumw(C, P, t, Cv);
    const int64_t Pp = part_size(P), S = sub_stride(P), ns = sub_per_part(P);
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        const int64_t e = t * kTile + 4 * (int64_t)threadIdx.x + m;
        if (e >= P) break;
        const int64_t x = e / Pp, local = e - x * Pp, end = min((x + 1) * Pp, P);
        if ((local + 1) % S == 0 || e == end - 1) ws.sub[x * ns + local / S] = Cv[m];
    }
    // The part of each of the tile's draws [t kTile, (t+1) kTile) (two Philox
    // blocks per thread): part y holds C' in [B_{y Pp / kTile - 1}, the next
    // part's bound), so the search reads one byte per draw instead of redrawing.
    const double W = ws.h->W, capW = below(W);
    const int parts = (int)((P + Pp - 1) / Pp);
    double lo[kParts];
#pragma unroll
    for (int y = 1; y < kParts; ++y)
        lo[y] = y < parts ? ws.bound[y * Pp / kTile - 1] : (double)INFINITY;
    uint32_t ids = 0;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int64_t q = t * (kTile / 2) + 2 * (int64_t)threadIdx.x + h;  // draws 2q, 2q+1
        const Block4 b = philox(seed, (uint32_t)q, instance, 0u, kTagMultinomial);
        const double x[2] = {fmin(unit53(b.r0, b.r1) * W, capW), fmin(unit53(b.r2, b.r3) * W, capW)};
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            uint32_t y = 0;
#pragma unroll
            for (int z = 1; z < kParts; ++z) y += lo[z] <= x[k] ? 1u : 0u;
            ids |= y << (8 * (2 * h + k));
        }
    }
    if (t * kTile + 4 * (int64_t)threadIdx.x < P)  // the array has 16 bytes of slack past P
        reinterpret_cast<uint32_t *>(ws.part + t * kTile)[threadIdx.x] = ids;
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

// Launch 4m: kParts x K blocks of 1024 threads; blocks b = x, x + kParts, ...
// serve part x (the draws whose ancestor lies in it), so with the round-robin
// placement of blocks on the XCDs one XCD searches one part and its slice of
// C stays in that XCD's L2. A block scans the part bytes of its share of the
// draws in chunks (16 per thread), queues the draws of its part in LDS
// (wave-aggregated slots), then every thread takes queued draws, redraws x,
// bisects the part's group ends staged in LDS and reads the group's 16 C'
// (one 128-byte line, up to 2^20 particles) with eight 16-byte loads.
constexpr int kSearchThreads = 1024;
constexpr int kIdsPerThread = 16;
constexpr int kQueue = kSearchThreads * kIdsPerThread;

__device__ __forceinline__ double multinomial_draw(uint64_t seed, uint32_t instance, int64_t i,
                                                   double W, double capW)
{
    const Block4 b = philox(seed, (uint32_t)(i >> 1), instance, 0u, kTagMultinomial);
    const double u = (i & 1) ? unit53(b.r2, b.r3) : unit53(b.r0, b.r1);
    return fmin(u * W, capW);
}

// First k in [0, n) with a[k] > x, given a[n - 1] > x (LDS, n < 2^31).
__device__ __forceinline__ int first_above_lds(const double *a, int n, double x)
{
    int base = 0;
    while (n > 1) {
        const int half = n >> 1;
        base = a[base + half - 1] <= x ? base + half : base;
        n -= half;
    }
    return base;
}

__global__ __launch_bounds__(kSearchThreads) void multinomial_search_kernel(
    const double *__restrict__ C, int32_t *__restrict__ anc, int64_t P, uint64_t seed,
    uint32_t instance, char *ws_raw, Rows rows)
{
    extern __shared__ double sh_sub[];
    __shared__ int32_t sh_queue[kQueue];
    __shared__ int32_t sh_count[2];
    const WsView ws = ws_view(ws_raw, P);
    const int part = (int)(blockIdx.x % kParts);
    const int64_t rank = blockIdx.x / kParts, K = gridDim.x / kParts;
    const int64_t Pp = part_size(P), S = sub_stride(P), ns = sub_per_part(P);
    const int64_t start = part * Pp, end = min(start + Pp, P);
    // this block's draws [d0, d1), a multiple of 16 wide
    const int64_t span = ((P + K - 1) / K + kIdsPerThread - 1) / kIdsPerThread * kIdsPerThread;
    const int64_t d0 = min(P, rank * span), d1 = min(P, d0 + span);
    const int flags = ws.h->flags;
    if (flags) {  // identity, written by the blocks of part 0
        if (part == 0) {
            for (int64_t i = d0 + threadIdx.x; i < d1; i += kSearchThreads) {
                anc[i] = (int32_t)i;
                if (rows.x_in) copy_row(rows, i, i, 0, 1);
            }
        }
        return;
    }
    if (start >= P) return;  // fewer tiles than parts
    const int groups = (int)((end - start + S - 1) / S);
    for (int k = threadIdx.x; k < groups; k += kSearchThreads) sh_sub[k] = ws.sub[part * ns + k];
    if (threadIdx.x == 0) {
        sh_count[0] = 0;
        sh_count[1] = 0;
    }
    const double W = ws.h->W, capW = below(W);
    const bool vec = S == 16 && (((uintptr_t)C) & 15) == 0;
    __syncthreads();
    const int lane = lane_id();
    int parity = 0;
    for (int64_t c0 = d0; c0 < d1; c0 += kQueue) {
        // (1) this thread's 16 part bytes; bit b of keep marks draw i0 + b as ours
        const int64_t i0 = c0 + (int64_t)kIdsPerThread * threadIdx.x;
        uint32_t keep = 0;
        if (i0 < d1) {
            const uint4 v = *reinterpret_cast<const uint4 *>(ws.part + i0);
            const uint32_t w4[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int b = 0; b < kIdsPerThread; ++b)
                if (i0 + b < d1 && ((w4[b >> 2] >> (8 * (b & 3))) & 0xffu) == (uint32_t)part)
                    keep |= 1u << b;
        }
        // (2) queue slots: a wave-wide prefix of the counts, one LDS atomic per wave
        const int cnt = __popc(keep);
        int incl = cnt;
#pragma unroll
        for (int off = 1; off < kWave; off <<= 1) {
            const int y = __shfl_up(incl, off, kWave);
            if (lane >= off) incl += y;
        }
        int base = 0;
        if (lane == kWave - 1) base = atomicAdd(&sh_count[parity], incl);
        base = __shfl(base, kWave - 1, kWave);
        int pos = base + incl - cnt;
        while (keep) {
            const int bit = __ffs((int)keep) - 1;
            keep &= keep - 1;
            sh_queue[pos++] = (int32_t)(i0 + bit);
        }
        __syncthreads();
        const int n = sh_count[parity];
        if (threadIdx.x == 0) sh_count[parity ^ 1] = 0;  // the next chunk's counter
        // (3) search the queued draws, two per thread at a time
        for (int idx = threadIdx.x; idx < n; idx += 2 * kSearchThreads) {
            int64_t i[2], j[2];
            bool on[2];
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                const int at = idx + k * kSearchThreads;
                on[k] = at < n;
                i[k] = on[k] ? sh_queue[at] : sh_queue[idx];
            }
            double x[2];
#pragma unroll
            for (int k = 0; k < 2; ++k) x[k] = multinomial_draw(seed, instance, i[k], W, capW);
            int64_t gbase[2], len[2];
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                gbase[k] = start + (int64_t)first_above_lds(sh_sub, groups, x[k]) * S;
                len[k] = min(S, end - gbase[k]);
            }
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                if (vec && len[k] == 16) {  // the whole line: count the C' <= x
                    const double2 *g2 = reinterpret_cast<const double2 *>(C + gbase[k]);
                    double2 c[8];
#pragma unroll
                    for (int h = 0; h < 8; ++h) c[h] = g2[h];
                    int below_x = 0;
#pragma unroll
                    for (int h = 0; h < 8; ++h)
                        below_x += (c[h].x <= x[k] ? 1 : 0) + (c[h].y <= x[k] ? 1 : 0);
                    j[k] = gbase[k] + below_x;
                } else {
                    j[k] = gbase[k] + first_above(C + gbase[k], len[k], x[k]);
                }
            }
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                if (on[k]) {
                    anc[i[k]] = (int32_t)j[k];
                    if (rows.x_in) copy_row(rows, i[k], j[k], 0, 1);
                }
            }
        }
        __syncthreads();  // the queue is free again
        parity ^= 1;
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
        if (const int rc = launch_fill<kStratified>(lw, anc, off, P, seed, instance, cumw, w, status,
                                                    stream, rows))
            return rc;
        break;
    case kSystematic:
        if (const int rc = launch_fill<kSystematic>(lw, anc, off, P, seed, instance, cumw, w, status,
                                                    stream, rows))
            return rc;
        break;
    case kMultinomial: {
        double *C = cumw ? cumw : reinterpret_cast<double *>(w + ws_layout(P, true).cumw);
        if (const int rc = launch_table<kMultinomial>(P, seed, instance, w, status, nullptr, stream))
            return rc;
        hipLaunchKernelGGL(cumulative_kernel, dim3((uint32_t)n), tb, 0, stream, lw, P, C, w, seed,
                           instance);
        const size_t smem = (size_t)sub_per_part(P) * sizeof(double);
        if (allow_dynamic_lds(reinterpret_cast<const void *>(&multinomial_search_kernel), smem))
            return -3;
        // K blocks per part: one per CU of an XCD at most, a chunk each at least
        int64_t K = (P + kQueue - 1) / kQueue;
        K = K < 1 ? 1 : (K > 32 ? 32 : K);
        const int64_t grid = kParts * K;
        hipLaunchKernelGGL(multinomial_search_kernel, dim3((uint32_t)grid), dim3(kSearchThreads),
                           smem, stream, C, anc, P, seed, instance, w, rows);
        break;
    }
    default:
        return -1;
    }
    return launch_status();
}

__global__ void workspace_lse_kernel(const char *ws_raw, int64_t P, double *out)
{
    if (threadIdx.x == 0) *out = ws_view(const_cast<char *>(ws_raw), P).h->lse;
}

int launch_workspace_lse(const void *ws, int64_t P, double *out, hipStream_t stream)
{
    hipLaunchKernelGGL(workspace_lse_kernel, dim3(1), dim3(64), 0, stream,
                       static_cast<const char *>(ws), P, out);
    return launch_status();
}

int launch_adaptive_B(const float *lw, int64_t P, double eps, uint32_t B_max, void *ws,
                      uint32_t *B_used, int32_t *status, hipStream_t stream)
{
    char *w = static_cast<char *>(ws);
    hipLaunchKernelGGL(tile_reduce_kernel, dim3((uint32_t)num_tiles(P)), dim3(kTileThreads), 0,
                       stream, lw, P, w);
    if (const int rc = launch_table<kAdaptiveB>(P, 0, 0u, w, status, nullptr, stream, eps, B_max,
                                                B_used))
        return rc;
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
    if (const int rc = launch_table<kLogSumExp>(P, 0, 0u, w, status, out, stream)) return rc;
    return launch_status();
}

}  // namespace rs
