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
//  2. table_kernel (up to 64 blocks): the tile sums rescaled to the global
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
// LDS, then one 128-byte line of C). Up to 1024 tiles the cumulative blocks
// rebuild the boundaries themselves (no table launch); up to two tiles one
// block does the whole multinomial resampling in one launch.
//
// Rounding: inside a tile C'_j = min(B_{t-1} + L_j, B_t), where L_j is a
// zero-weight-aware running maximum of the tile's scan, and C'_j = B_t from
// the tile's last positive weight on. This keeps C' non-decreasing across
// tiles although the tile sums and the in-tile scans round differently, and
// keeps zero-weight particles unselectable. C' agrees with the binary64
// left-to-right sum to a few ulps.
#include <hip/hip_runtime.h>

#include <atomic>
#include <mutex>

#include "common.h"
#include "launch.h"
#include "prefix.h"
#include "prefix_impl.h"
#include "resample.h"

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

template <int KIND, bool LDS, int NT>
__global__ __launch_bounds__(NT) void table_kernel(int64_t P, uint64_t seed, uint32_t instance,
                                                   char *ws_raw, int32_t *status, double *lse_out,
                                                   double eps, uint32_t B_max, uint32_t *B_used)
{
    extern __shared__ double sh_tab[];  // [n] boundaries, then the block's counts
    const WsView ws = ws_view(ws_raw, P);
    const int64_t n = num_tiles(P);
    double *bound = LDS ? sh_tab : ws.bound;
    int32_t *count = LDS ? reinterpret_cast<int32_t *>(sh_tab + n) : ws.count;
    table_body<KIND, NT>(P, seed, instance, ws_raw, status, lse_out, bound, count, eps, B_max,
                         B_used, blockIdx.x, gridDim.x);
}

// Stratified/systematic tables with LDS boundaries split the counts over up
// to kTableParts blocks (one count per thread up to 2^24 particles); the
// rest run one block. The split changes no result: each block rebuilds the same
// boundaries and the counts are exact.
constexpr int64_t kTableParts = 64;

// Beyond 1024 tiles the table blocks run kTableWideThreads threads: the
// element-wise passes and the counts spread over two waves per SIMD, while
// the runs and their scans stay with the first kTileThreads threads, so the
// boundaries are the same sums. (At 1024 threads the 128-register cap puts
// the passes' arrays in scratch memory.)
constexpr int kTableWideThreads = 512;

template <int KIND, int NT>
int launch_table_nt(int64_t P, uint64_t seed, uint32_t instance, char *w, int32_t *status,
                    double *lse_out, hipStream_t stream, double eps, uint32_t B_max,
                    uint32_t *B_used)
{
    const int64_t n = num_tiles(P);
    if (n <= kTableLdsTiles) {
        int64_t parts = 1;
        if (KIND == kStratified || KIND == kSystematic) {
            // at most NT - 1 tiles a block: with the one before its first
            // tile, every thread then has at most one count
            parts = (n + NT - 2) / (NT - 1);
            parts = parts > kTableParts ? kTableParts : parts;
        }
        // a block's counts (one extra); only stratified and systematic count
        const bool counts = KIND == kStratified || KIND == kSystematic;
        const int64_t slice = counts ? (n + parts - 1) / parts + 2 : 0;
        const size_t smem = (size_t)n * sizeof(double) + (size_t)slice * sizeof(int32_t);
        if (allow_dynamic_lds(reinterpret_cast<const void *>(&table_kernel<KIND, true, NT>), smem))
            return -3;
        hipLaunchKernelGGL((table_kernel<KIND, true, NT>), dim3((uint32_t)parts), dim3(NT), smem,
                           stream, P, seed, instance, w, status, lse_out, eps, B_max, B_used);
    } else {
        hipLaunchKernelGGL((table_kernel<KIND, false, NT>), dim3(1), dim3(NT), 0, stream, P, seed,
                           instance, w, status, lse_out, eps, B_max, B_used);
    }
    return 0;
}

template <int KIND>
int launch_table(int64_t P, uint64_t seed, uint32_t instance, char *w, int32_t *status,
                  double *lse_out, hipStream_t stream, double eps = 0.0, uint32_t B_max = 0,
                  uint32_t *B_used = nullptr)
{
    if (num_tiles(P) > (int64_t)kTileThreads * kRegTiles)
        return launch_table_nt<KIND, kTableWideThreads>(P, seed, instance, w, status, lse_out,
                                                        stream, eps, B_max, B_used);
    return launch_table_nt<KIND, kTileThreads>(P, seed, instance, w, status, lse_out, stream, eps,
                                               B_max, B_used);
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

// ------------------------------------------------------ one-pass fill
// Stratified/systematic resampling in one launch (P <= 2^20; the launcher
// enqueues a small fill kernel before it): the three phases of the launches
// above (tile reduction, boundaries and counts, fill) with the grid-wide step
// done inside the kernel. Block b owns tiles b and
// b + G (G = gridDim.x = ceil(n / 2)). It loads their log-weights (and, with
// DS > 0, their state rows) once, reduces each tile exactly as
// tile_reduce_body does and publishes (max, sum, flags) as three 64-bit words
// per tile, each carrying a 32-bit tag in its high half. The block then reads
// every tile's words back, runs the same boundaries code as the table launch
// on them (so every block holds the same bits the three-launch path computes)
// and fills its own tiles from registers and LDS, plus the overflow windows
// of heavy tiles it is assigned.
//
// No release fence is needed: each word is self-contained, written and read
// with relaxed device-scope atomics, which go to the point of coherence
// shared by the eight XCDs (no L2 write-back). The launcher clears the 3n
// words with a fill kernel ordered before this one, and a published word's
// high half, pub_tag(t, k), is never zero: every word that passes the test
// was written by this call, whatever earlier calls (of any kind or size)
// left in the workspace, and replays of a captured graph clear them again.
// The wait is bounded: a block that has not seen a tile's words after
// wait_ticks of the real-time clock reduces that tile itself (the same
// function, the same bits), so the results never depend on all blocks being
// resident at once; only the speed does.
__device__ __forceinline__ uint32_t pub_tag(int64_t t, int k)
{
    return (uint32_t)(3 * t + k) + 1u;  // the word's index plus one (3n < 2^32)
}

// Word 0 of a tile: its max as binary32 bits, or, when the tile holds a NaN
// or +inf log-weight, a quiet NaN whose payload is the flags (a clean tile's
// max is never NaN).
__device__ __forceinline__ uint32_t pub_max_word(float mx, int fl)
{
    return fl ? (0x7FC00000u | (uint32_t)fl) : __float_as_uint(mx);
}

__device__ __forceinline__ int pub_flags(uint32_t w0)
{
    const bool nan = (w0 & 0x7F800000u) == 0x7F800000u && (w0 & 0x007FFFFFu) != 0u;
    return nan ? (int)(w0 & 0xFFu) : 0;
}

constexpr int kOnePassWindows = 4;  // overflow windows per block at most

template <int KIND, int DS>
__global__ __launch_bounds__(kTileThreads) void onepass_kernel(
    const float *__restrict__ lw, int32_t *__restrict__ anc, int32_t *__restrict__ off, int64_t P,
    uint64_t seed, uint32_t instance, double *cumw, char *ws_raw, int32_t *status, Rows rows,
    uint64_t wait_ticks)
{
    // Cs (the fill's cumulative weights) and sh_bound (the tile boundaries) in
    // one array: before the boundaries it holds the tiles' payloads
    __shared__ double lds_cb[kTile + kOnePassMaxTiles];
    double *Cs = lds_cb, *sh_bound = lds_cb + kTile;
    static_assert(3 * kOnePassMaxTiles * sizeof(uint32_t) <= sizeof(lds_cb), "payloads fit");
    static_assert(kOnePassMaxTiles * (sizeof(int32_t) + 1) <= kChunk * sizeof(int32_t),
                  "the missing-tile list and bytes fit in sh_anc");
    __shared__ int32_t sh_anc[kChunk];
    __shared__ int64_t sh_cnt[2 * kOnePassTiles];        // lo, hi of the block's tiles
    __shared__ int64_t sh_win[kOnePassWindows][3];       // owner tile (-1: none), lo, hi
    __shared__ int sh_nmiss;
    extern __shared__ float4 sh_rows4[];  // DS > 0: the block's tiles' rows, kTile x DS floats each
    constexpr int kRow4 = kTile * (DS > 0 ? DS : 1) / 4;  // float4 per tile of rows
    static_assert(kTile / 4 == kTileThreads, "one float4 of rows per thread and DS");

    const WsView ws = ws_view(ws_raw, P);
    const WsLayout L = ws_layout(P, false);
    uint64_t *pub = reinterpret_cast<uint64_t *>(ws_raw + L.pub);
    const int64_t n = num_tiles(P), G = gridDim.x, b = blockIdx.x;
    const int tid = threadIdx.x;

    // every load of the block's own data is issued before the first wait
    float v[kOnePassTiles][4];
#pragma unroll
    for (int r = 0; r < kOnePassTiles; ++r) {
        const int64_t t = b + r * G;
        if (t < n) load_tile4(lw, P, t, v[r]);
        else v[r][0] = v[r][1] = v[r][2] = v[r][3] = -INFINITY;
    }
    float4 xs[kOnePassTiles][DS > 0 ? DS : 1];
    if (DS > 0) {
        const int64_t total = P * DS;  // floats of state
#pragma unroll
        for (int r = 0; r < kOnePassTiles; ++r) {
            const int64_t t = b + r * G;
#pragma unroll
            for (int q = 0; q < DS; ++q) {
                const int64_t el = t * kTile * DS + 4 * (int64_t)(q * kTileThreads + tid);
                float4 x = make_float4(0.f, 0.f, 0.f, 0.f);
                if (t < n) {
                    if (el + 4 <= total) {
                        x = *reinterpret_cast<const float4 *>(rows.x_in + el);
                    } else {
                        if (el + 0 < total) x.x = rows.x_in[el + 0];
                        if (el + 1 < total) x.y = rows.x_in[el + 1];
                        if (el + 2 < total) x.z = rows.x_in[el + 2];
                    }
                }
                xs[r][q] = x;
            }
        }
    }

    // ------------------------------------------------ reduce and publish
#pragma unroll
    for (int r = 0; r < kOnePassTiles; ++r) {
        const int64_t t = b + r * G;
        if (t >= n) break;  // uniform
        float mx;
        double s;
        int fl;
        tile_reduce_vals(v[r], &mx, &s, &fl);
        if (tid == 0) {
            const uint64_t sb = (uint64_t)__double_as_longlong(s);
            uint64_t *w = pub + 3 * t;
            __hip_atomic_store(w + 0, ((uint64_t)pub_tag(t, 0) << 32) | pub_max_word(mx, fl),
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(w + 1, ((uint64_t)pub_tag(t, 1) << 32) | (sb >> 32),
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(w + 2, ((uint64_t)pub_tag(t, 2) << 32) | (sb & 0xFFFFFFFFu),
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
    if (DS > 0) {
#pragma unroll
        for (int r = 0; r < kOnePassTiles; ++r)
#pragma unroll
            for (int q = 0; q < DS; ++q) sh_rows4[r * kRow4 + q * kTileThreads + tid] = xs[r][q];
    }

    // ------------------------------------------------ every tile's values
    // The 3n words are read as one flat array, 256 consecutive words per
    // pass of the block (coalesced), and their payloads collected in LDS
    // (the space of Cs and sh_bound, free until the boundaries); each thread
    // then takes its own run of tiles from there.
    constexpr int kPolls = 3 * kOnePassMaxTiles / kTileThreads;  // words per thread at most
    static_assert(kPolls <= 32, "one mask bit per word");
    uint32_t *pay = reinterpret_cast<uint32_t *>(lds_cb);  // 3n payloads
    const int64_t nw = 3 * n;
    uint32_t need = 0, tag[kPolls];
#pragma unroll
    for (int i = 0; i < kPolls; ++i) {
        const int64_t w = tid + (int64_t)i * kTileThreads;
        tag[i] = 0;
        if (w < nw) {
            need |= 1u << i;
            tag[i] = pub_tag(w / 3, (int)(w % 3));
        }
    }
    const uint64_t start = wall_clock64();
    bool late = false;
    while (true) {
        uint64_t got[kPolls];
#pragma unroll
        for (int i = 0; i < kPolls; ++i)
            if (need & (1u << i))
                got[i] = __hip_atomic_load(pub + tid + i * kTileThreads, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
#pragma unroll
        for (int i = 0; i < kPolls; ++i) {
            if ((need & (1u << i)) && (uint32_t)(got[i] >> 32) == tag[i]) {
                pay[tid + i * kTileThreads] = (uint32_t)got[i];
                need &= ~(1u << i);
            }
        }
        if (!__syncthreads_or(need != 0u)) break;
        if (__syncthreads_or(tid == 0 && wall_clock64() - start > wait_ticks)) {
            late = true;
            break;
        }
        __builtin_amdgcn_s_sleep(2);
    }
    if (late) {
        // reduce the tiles with a word still missing here (the same function,
        // so the same values); sh_anc holds the list, then a byte per tile
        uint8_t *miss = reinterpret_cast<uint8_t *>(sh_anc + kOnePassMaxTiles);
        for (int64_t t = tid; t < n; t += kTileThreads) miss[t] = 0;
        if (tid == 0) sh_nmiss = 0;
        __syncthreads();
#pragma unroll
        for (int i = 0; i < kPolls; ++i)
            if (need & (1u << i)) miss[(tid + i * kTileThreads) / 3] = 1;
        __syncthreads();
        for (int64_t t = tid; t < n; t += kTileThreads)
            if (miss[t]) sh_anc[atomicAdd(&sh_nmiss, 1)] = (int32_t)t;
        __syncthreads();
        const int nm = sh_nmiss;
        for (int i = 0; i < nm; ++i) {
            const int64_t t = sh_anc[i];
            float vv[4];
            load_tile4(lw, P, t, vv);
            float mx;
            double s;
            int fl;
            tile_reduce_vals(vv, &mx, &s, &fl);
            if (tid == 0) {
                const uint64_t sb = (uint64_t)__double_as_longlong(s);
                pay[3 * t] = pub_max_word(mx, fl);
                pay[3 * t + 1] = (uint32_t)(sb >> 32);
                pay[3 * t + 2] = (uint32_t)sb;
            }
        }
    }
    __syncthreads();
    int64_t t0, t1;
    bool reg;
    tile_run(n, &t0, &t1, &reg);  // reg: n <= 1024
    float mt[kRegTiles];
    double S[kRegTiles];
    int fl = 0;
    float m = -INFINITY;
#pragma unroll
    for (int k = 0; k < kRegTiles; ++k) {
        mt[k] = -INFINITY;
        S[k] = 0.0;
        const int64_t t = t0 + k;
        if (t < t1) {
            const uint32_t w0 = pay[3 * t];
            mt[k] = __uint_as_float(w0);
            fl |= pub_flags(w0);
            S[k] = __longlong_as_double(
                (long long)(((uint64_t)pay[3 * t + 1] << 32) | (uint64_t)pay[3 * t + 2]));
        }
        m = fmaxf(m, mt[k]);
    }
    __syncthreads();  // sh_bound (part of the payload space) is written below
    const TableSums sums = boundaries_tail<false>(ws, n, t0, t1, true, fl, m, mt, S, sh_bound);
    if (b == 0 && tid == 0) {
        WsHeader *h = ws.h;
        h->flags = sums.flags;
        h->m = sums.m;
        h->W = sums.W;
        h->delta = sums.W / (double)P;
        h->lse = sums.flags
                     ? ((sums.flags & (kFlagNan | kFlagPosInf)) ? (double)NAN : -(double)INFINITY)
                     : (double)sums.m + log(sums.W);
        if (sums.flags) raise_flags(status, sums.flags);
    }
    if (sums.flags) {  // flagged input: identity ancestors and rows, one offspring each
        for (int r = 0; r < kOnePassTiles; ++r) {
            const int64_t t = b + r * G;
            for (int64_t j = t * kTile + tid; j < min(P, (t + 1) * kTile); j += kTileThreads) {
                if (anc) anc[j] = (int32_t)j;
                if (off) off[j] = 1;
                if (cumw) cumw[j] = (double)NAN;
                if (rows.x_in)
                    for (int d = 0; d < rows.D; ++d)
                        rows.x_out[j * rows.D + d] = rows.x_in[j * rows.D + d];
            }
        }
        return;
    }
    const double W = sums.W, delta = W / (double)P;
    const float mg = sums.m;  // the largest log-weight (m above is this thread's run's)
    const double u_sys = KIND == kSystematic ? systematic_offset(seed, instance) : 0.0;

    // ------------------------------------------------ draw counts
    // the block's tiles: N(B_{t-1}) and N(B_t) on four waves at once
    const int wave = tid / kWave, lane = tid % kWave;
    if (lane == 0) {
        const int r = wave / 2;
        const int64_t t = b + r * G;
        if (r < kOnePassTiles && t < n) {
            const int64_t c = (wave & 1) ? t : t - 1;
            sh_cnt[wave] = c < 0 ? 0
                                 : count_below<KIND>(sh_bound[c], P, W, delta, seed, instance,
                                                     u_sys);
        }
    }
    // overflow windows q = b, b + G, ...: only the tile holding the window's
    // first draw can own it, and only when more than kChunk - 3 draws fall in
    // that tile (N(B_t) - N(B_{t-1}) <= (B_t - B_{t-1}) / delta + 2, so tiles
    // far below that bound are skipped without counting)
    const int64_t nwin = num_windows(P);
    if (lane == 32 && wave < kOnePassWindows) {
        const int64_t q = b + wave * G;
        int64_t owner = -1, lo_t = 0, hi_t = 0;
        if (q < nwin) {
            const double x0 = draw_point<KIND>(q * kWindow, delta, seed, instance, u_sys);
            const int64_t tt = first_bound_above(sh_bound, n, fmin(x0, below(W)));
            const double Blo = tt > 0 ? sh_bound[tt - 1] : 0.0;
            if ((sh_bound[tt] - Blo) / delta + 8.0 > (double)(kChunk - 3)) {
                hi_t = count_below<KIND>(sh_bound[tt], P, W, delta, seed, instance, u_sys);
                lo_t = tt > 0 ? count_below<KIND>(Blo, P, W, delta, seed, instance, u_sys) : 0;
                const int64_t M = (lo_t & ~(int64_t)3) + kChunk;
                if (max(q * kWindow, M) < min((q + 1) * kWindow, hi_t)) owner = tt;
            }
        }
        sh_win[wave][0] = owner;
        sh_win[wave][1] = lo_t;
        sh_win[wave][2] = hi_t;
    }
    __syncthreads();

    // ------------------------------------------------ fill the block's tiles
    for (int r = 0; r < kOnePassTiles; ++r) {
        const int64_t t = b + r * G;
        if (t >= n) break;  // uniform
        const int64_t lo = sh_cnt[2 * r], hi = sh_cnt[2 * r + 1];
        const int64_t a0 = lo & ~(int64_t)3, oe = min(hi, a0 + kChunk);
        if (lo >= oe && !cumw && !off) continue;  // no draws and nothing else to write
        double wts[4];
        tile_weights(v[r], mg, wts);
        const float *staged = DS > 0 ? reinterpret_cast<const float *>(sh_rows4 + r * kRow4)
                                     : nullptr;
        fill_chunk<KIND>(anc, off, P, seed, instance, cumw, true, t, lo, oe, a0, lo, hi,
                         t > 0 ? sh_bound[t - 1] : 0.0, sh_bound[t], W, wts, rows.x_in,
                         rows.x_out, rows.D, status, Cs, sh_anc, staged);
        __syncthreads();  // Cs and sh_anc are reused
    }
    // ------------------------------------------------ overflow windows owned
    for (int k = 0; k < kOnePassWindows; ++k) {
        const int64_t t = sh_win[k][0];
        if (t < 0) continue;  // uniform
        const int64_t q = b + k * G, lo = sh_win[k][1], hi = sh_win[k][2];
        const int64_t ob = max(q * kWindow, (lo & ~(int64_t)3) + kChunk);
        const int64_t oe = min((q + 1) * kWindow, hi), a0 = ob & ~(int64_t)3;
        float vv[4];
        double wts[4];
        load_tile4(lw, P, t, vv);
        tile_weights(vv, mg, wts);
        fill_chunk<KIND>(anc, off, P, seed, instance, cumw, false, t, ob, oe, a0, lo, hi,
                         t > 0 ? sh_bound[t - 1] : 0.0, sh_bound[t], W, wts, rows.x_in,
                         rows.x_out, rows.D, status, Cs, sh_anc, nullptr);
        __syncthreads();
    }
}

// Guide table of the multinomial search (Chen and Asau's method for
// inverse-CDF sampling). Part x's C' range [lo, hi] (lo = C' before the part,
// hi = its last C', both tile boundaries) is cut into nb = groups equal
// buckets; bucket(v) = floor((v - lo) nb / (hi - lo)) clamped to [0, nb).
// Each step is monotone in v (rounded subtraction, product by a non-negative
// scale, clamp), so v <= v' gives bucket(v) <= bucket(v'): the guide's
// bounds below rest on that, not on the buckets being exactly equal. Every
// kernel derives the buckets from the same bound entries, bit for bit.
struct Buckets {
    double base, scale;
    int nb;
    __device__ __forceinline__ int of(double v) const
    {
        const double f = (v - base) * scale;
        return f >= (double)nb ? nb - 1 : (f > 0.0 ? (int)f : 0);
    }
};

// Part x's bounds in C': lo = C' before its first particle, hi = its last C'.
__device__ __forceinline__ void part_range(const double *bound, int64_t P, int part, double *lo,
                                           double *hi)
{
    const int64_t Pp = part_size(P), start = part * Pp, end = min(start + Pp, P);
    *lo = start > 0 ? bound[start / kTile - 1] : 0.0;
    *hi = bound[(end - 1) / kTile];
}

__device__ __forceinline__ Buckets make_buckets(double lo, double hi, int nb)
{
    Buckets bk;
    bk.nb = nb;
    bk.base = lo;
    const double width = hi - lo;
    double scale = (width > 0.0 && width < (double)INFINITY) ? (double)nb / width : 0.0;
    if (!(scale < (double)INFINITY)) scale = 0.0;
    bk.scale = scale;
    return bk;
}

// guide[q] = v for q in [from, to), 16-byte stores where aligned (a group
// holding much of the part's weight spans many buckets).
__device__ __forceinline__ void fill_guide(uint16_t *guide, int from, int to, uint16_t v)
{
    int q = from;
    for (; q < to && (q & 7); ++q) guide[q] = v;
    const uint32_t v2 = (uint32_t)v * 0x10001u;
    const uint4 v8 = make_uint4(v2, v2, v2, v2);
    for (; q + 8 <= to; q += 8) *reinterpret_cast<uint4 *>(guide + q) = v8;
    for (; q < to; ++q) guide[q] = v;
}

// ------------------------------------------------------ multinomial
// Launch 3m: one block per tile writes C' for the tile; into ws.sub the last
// C' of every sub_stride(P)-particle group of each part (the last group of a
// part ends at the part's end) and the guide entries those groups own; and
// the part byte of each of the tile's draws.
// Up to this many tiles the cumulative blocks rebuild the boundaries themselves.
constexpr int64_t kFusedCumulativeTiles = 1024;

// With FUSED (at most kFusedCumulativeTiles tiles) there is no table launch: every
// block rebuilds the tile boundaries in LDS from the tile sums (the same
// function and order as the table launch, so the same bits), writes its own
// tile's boundary for the search, and block 0 writes the header.
template <bool FUSED>
__global__ __launch_bounds__(kTileThreads) void cumulative_kernel(const float *__restrict__ lw,
                                                                  int64_t P, double *C,
                                                                  char *ws_raw, uint64_t seed,
                                                                  uint32_t instance,
                                                                  int32_t *status)
{
    __shared__ double Cs[kTile];
    __shared__ double sh_bound[FUSED ? kFusedCumulativeTiles : 1];
    const WsView ws = ws_view(ws_raw, P);
    const int64_t t = blockIdx.x;
    float v[4];
    load_tile4(lw, P, t, v);
    int flags;
    float m;
    double W;
    const double *bound = ws.bound;
    if (FUSED) {
        const TableSums sums = boundaries<false>(ws, P, sh_bound);
        flags = sums.flags;
        m = sums.m;
        W = sums.W;
        bound = sh_bound;
        if (threadIdx.x == 0) {
            if (!flags) ws.bound[t] = sh_bound[t];
            if (t == 0) {
                WsHeader *h = ws.h;
                h->flags = flags;
                h->m = m;
                h->W = W;
                h->delta = W / (double)P;
                h->lse = flags ? ((flags & (kFlagNan | kFlagPosInf)) ? (double)NAN
                                                                     : -(double)INFINITY)
                               : (double)m + log(W);
                if (flags) raise_flags(status, flags);
            }
        }
    } else {
        flags = ws.h->flags;
        m = ws.h->m;
        W = ws.h->W;
    }
    // Every boundary this block needs is read before the flags are tested
    // (all reads stay inside the arrays; the values are used only when the
    // flags are clear), so the reads overlap instead of following each other.
    const int64_t Pp = part_size(P), S = sub_stride(P), ns = sub_per_part(P);
    const int xt = (int)(t * kTile / Pp);  // a part is whole tiles
    const int parts = (int)((P + Pp - 1) / Pp);
    const double Blo = t > 0 ? bound[t - 1] : 0.0, Bhi = bound[t];
    double plo, phi;
    part_range(bound, P, xt, &plo, &phi);
    double lo[kParts];
#pragma unroll
    for (int y = 1; y < kParts; ++y)
        lo[y] = y < parts ? bound[y * Pp / kTile - 1] : (double)INFINITY;
    if (flags) {
        const int64_t base = t * kTile + 4 * (int64_t)threadIdx.x;
        for (int k = 0; k < 4; ++k)
            if (base + k < P) C[base + k] = (double)NAN;
        return;
    }
    double w[4], Cv[4];
    tile_weights(v, m, w);
    tile_cumulative(w, Blo, Bhi, Cs, Cv);
    store_cumw(C, P, t, Cv);
    // the group ends of this tile, and their guide entries: group g writes
    // guide[q] = g for the buckets q in (bucket(end[g - 1]), bucket(end[g])],
    // the part's last group also (bucket(end[last]), nb]; so guide[q] is the
    // first group whose end lies in bucket q or later and every entry is
    // written once. A group's predecessor end is in this tile's Cs or is an
    // earlier tile's last C', which equals that tile's bound bit for bit.
    const Buckets bk = make_buckets(plo, phi, (int)((min((xt + 1) * Pp, P) - xt * Pp + S - 1) / S));
    uint16_t *guide = ws.guide + xt * guide_stride(P);
#pragma unroll
    for (int mm = 0; mm < 4; ++mm) {
        const int64_t e = t * kTile + 4 * (int64_t)threadIdx.x + mm;
        if (e >= P) break;
        const int64_t local = e - xt * Pp, end = min((xt + 1) * Pp, P);
        if ((local + 1) % S == 0 || e == end - 1) {
            const int64_t g = local / S;
            ws.sub[xt * ns + g] = Cv[mm];
            const int bg = bk.of(Cv[mm]);
            int bp = -1;
            if (g > 0) {
                const int64_t pe = xt * Pp + g * S - 1;
                bp = bk.of(pe >= t * kTile ? Cs[pe - t * kTile] : bound[pe / kTile]);
            }
            if (bg > bp) fill_guide(guide, bp + 1, bg + 1, (uint16_t)g);
            if (e == end - 1) fill_guide(guide, max(bg, bp) + 1, bk.nb + 1, (uint16_t)g);
        }
    }
    // The part of each of the tile's draws [t kTile, (t+1) kTile) (two Philox
    // blocks per thread): part y holds C' in [B_{y Pp / kTile - 1}, the next
    // part's bound), so the search reads one byte per draw instead of redrawing.
    const double capW = below(W);
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
// C stays in that XCD's L2. A block stages in LDS the part's group ends
// (every S-th C') and the guide table the cumulative launch built over them
// (Chen and Asau's method for inverse-CDF sampling: the part's C' range is cut
// into as many equal buckets as there are groups, and guide[b] is the first
// group whose end falls in bucket b or later). It then scans the part bytes of its share of the draws in
// chunks (32 per thread), queues the draws of its part in LDS (wave-aggregated
// slots), and every thread takes queued draws, redraws x, bisects only the
// groups [guide[b], guide[b + 1]] of x's bucket (about one on average) and
// counts the group's 16 C' (one 128-byte line, up to 2^20 particles), eight
// lanes reading each line together.
constexpr int kSearchThreads = 1024;
constexpr int kIdsPerThread = 32;
constexpr int kQueue = kSearchThreads * kIdsPerThread;  // draws per chunk
static_assert(kQueue <= 65536, "queue entries are 16-bit offsets into the chunk");
constexpr int kSlots = 3;

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

// The 16 part bytes of draws [i0, i0 + 16), read unconditionally (from the
// array's start when i0 >= d1: the caller ignores bytes past d1), so the load
// stays in flight instead of being waited on at the end of a branch.
__device__ __forceinline__ uint4 load_part_bytes(const uint8_t *part, int64_t i0, int64_t d1)
{
    return *reinterpret_cast<const uint4 *>(part + (i0 < d1 ? i0 : 0));
}

// Orders a wave's LDS accesses around an exchange between its own lanes
// (the compiler keeps them in program order; the hardware runs one wave's
// LDS instructions in order).
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// For each lane's draw (x, gbase) with coop set: the number of the 16 C' of
// its group (one 128-byte line at C + gbase) that are <= x. Eight lanes read
// a line together, 16 bytes each, so one load instruction covers eight whole
// lines (the address unit then handles 8 lines per instruction, not 64); a
// ballot per comparison gives each owner its line's count. Group grp (lanes
// 8 grp .. 8 grp + 7) reads, in round r, the line of the draw owned by lane
// 8 r + grp. The draws reach their readers through the wave's 768-byte LDS
// exchange area (xw, gw): lane s writes to entry (s mod 8) * 8 + s / 8, so
// the eight draws a group reads lie together and come back in six 16-byte
// reads. Lanes without a cooperative draw read the line at C (the search runs
// only for P > 2048, so C[0..15] exists) and count nothing. Every lane of the
// wave must call this (lanes without a draw pass coop = false).
__device__ __forceinline__ int line_count_coop(const double *C, double x, int64_t gbase, bool coop,
                                               double *xw, int32_t *gw)
{
    const int lane = lane_id(), grp = lane >> 3, sub = lane & 7;
    const uint64_t coop_mask = __ballot(coop);
    wave_lds_sync();  // the previous call's reads are done
    xw[sub * 8 + grp] = x;
    gw[sub * 8 + grp] = coop ? (int32_t)gbase : 0;
    wave_lds_sync();
    double xs[8];
    int32_t gs[8];
    {
        const double2 *xv = reinterpret_cast<const double2 *>(xw + grp * 8);
        const int4 *gv = reinterpret_cast<const int4 *>(gw + grp * 8);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const double2 d = xv[q];
            xs[2 * q] = d.x;
            xs[2 * q + 1] = d.y;
        }
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int4 g = gv[q];
            gs[4 * q] = g.x, gs[4 * q + 1] = g.y, gs[4 * q + 2] = g.z, gs[4 * q + 3] = g.w;
        }
    }
    double2 c[8];
#pragma unroll
    for (int r = 0; r < 8; ++r) {
        const double2 v = reinterpret_cast<const double2 *>(C + gs[r])[sub];
        const bool cs = ((coop_mask >> (8 * r + grp)) & 1ull) != 0;
        c[r] = cs ? v : make_double2((double)INFINITY, (double)INFINITY);
    }
    int cnt = 0;
#pragma unroll
    for (int r = 0; r < 8; ++r) {
        const uint64_t m1 = __ballot(c[r].x <= xs[r]), m2 = __ballot(c[r].y <= xs[r]);
        if (grp == r)  // this lane owns the draw read by group sub in round r
            cnt = __popcll((m1 >> (8 * sub)) & 0xffull) + __popcll((m2 >> (8 * sub)) & 0xffull);
    }
    return cnt;
}

// WIDE: groups of more than one line (sub_stride(P) > 16, beyond 2^20
// particles); the one-line form carries no line-end step.
template <bool WIDE>
__global__ __launch_bounds__(kSearchThreads) void multinomial_search_kernel(
    const double *__restrict__ C, int32_t *__restrict__ anc, int64_t P, uint64_t seed,
    uint32_t instance, char *ws_raw, Rows rows)
{
    extern __shared__ double sh_sub[];
    __shared__ uint16_t sh_queue[kQueue];  // draw index - chunk start
    __shared__ __align__(16) uint16_t sh_guide[kSubMax + 8];
    static_assert(kSubMax % 8 == 0, "guide rows are whole 16-byte vectors");
    __shared__ int32_t sh_count[2];
    __shared__ __align__(16) double sh_xw[kSearchThreads];   // line_count_coop exchange,
    __shared__ __align__(16) int32_t sh_gw[kSearchThreads];  // 64 entries per wave
    const WsView ws = ws_view(ws_raw, P);
    const int part = (int)(blockIdx.x % kParts);
    const int64_t rank = blockIdx.x / kParts, K = gridDim.x / kParts;
    const int64_t Pp = part_size(P), S = sub_stride(P), ns = sub_per_part(P);
    const int64_t start = part * Pp, end = min(start + Pp, P);
    // this block's draws [d0, d1), a multiple of kIdsPerThread wide
    const int64_t span = ((P + K - 1) / K + kIdsPerThread - 1) / kIdsPerThread * kIdsPerThread;
    const int64_t d0 = min(P, rank * span), d1 = min(P, d0 + span);
    // every global read of the set-up is issued before the first wait: the
    // header, the first chunk's part bytes, the group ends (at most kSubMax,
    // 8 per thread) and the guide
    const int flags = ws.h->flags;
    const double W = ws.h->W, capW = below(W);
    const int groups = start < P ? (int)((end - start + S - 1) / S) : 0;
    double plo = 0.0, phi = 0.0;
    if (start < P) part_range(ws.bound, P, part, &plo, &phi);
    uint4 pv0 = load_part_bytes(ws.part, d0 + (int64_t)kIdsPerThread * threadIdx.x, d1);
    uint4 pv1 = load_part_bytes(ws.part, d0 + (int64_t)kIdsPerThread * threadIdx.x + 16, d1);
    constexpr int kStage = (int)(kSubMax / kSearchThreads);
    static_assert(kSubMax % kSearchThreads == 0, "whole staging rounds");
    double stage[kStage];
#pragma unroll
    for (int r = 0; r < kStage; ++r) {
        const int k = (int)threadIdx.x + r * kSearchThreads;
        stage[r] = k < groups ? ws.sub[part * ns + k] : 0.0;
    }
    // the part's guide: at most kSubMax + 8 entries, 16 bytes per thread and
    // one more vector for thread 0
    const int gv = start < P ? (int)(guide_stride(P) / 8) : 0;
    const uint4 *gsrc = reinterpret_cast<const uint4 *>(ws.guide + part * guide_stride(P));
    const uint4 g0v = (int)threadIdx.x < gv ? gsrc[threadIdx.x] : make_uint4(0u, 0u, 0u, 0u);
    const uint4 g1v = threadIdx.x == 0 && gv > kSearchThreads ? gsrc[kSearchThreads]
                                                            : make_uint4(0u, 0u, 0u, 0u);
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
#pragma unroll
    for (int r = 0; r < kStage; ++r) {
        const int k = (int)threadIdx.x + r * kSearchThreads;
        if (k < groups) sh_sub[k] = stage[r];
    }
    if ((int)threadIdx.x < gv) reinterpret_cast<uint4 *>(sh_guide)[threadIdx.x] = g0v;
    if (threadIdx.x == 0 && gv > kSearchThreads)
        reinterpret_cast<uint4 *>(sh_guide)[kSearchThreads] = g1v;
    if (threadIdx.x == 0) {
        sh_count[0] = 0;
        sh_count[1] = 0;
    }
    const bool vec = (((uintptr_t)C) & 15) == 0;  // S is a power of two >= 16
    __syncthreads();
    const Buckets bk = make_buckets(plo, phi, groups);
    const int lane = lane_id();
    int parity = 0;
    for (int64_t c0 = d0; c0 < d1; c0 += kQueue) {
        // (1) this thread's 32 part bytes; bit b of keep marks draw i0 + b as ours
        const int64_t i0 = c0 + (int64_t)kIdsPerThread * threadIdx.x;
        uint32_t keep = 0;
        {
            const uint32_t w8[8] = {pv0.x, pv0.y, pv0.z, pv0.w, pv1.x, pv1.y, pv1.z, pv1.w};
#pragma unroll
            for (int b = 0; b < kIdsPerThread; ++b)
                if (i0 + b < d1 && ((w8[b >> 2] >> (8 * (b & 3))) & 0xffu) == (uint32_t)part)
                    keep |= 1u << b;
        }
        // the next chunk's, while this one runs
        pv0 = load_part_bytes(ws.part, i0 + kQueue, d1);
        pv1 = load_part_bytes(ws.part, i0 + kQueue + 16, d1);
        // (2) queue slots: a wave-wide prefix of the counts, one LDS atomic per wave
        const int cnt = __popc(keep);
        const int incl = wave_scan(cnt, 0, AddOp{});
        int base = 0;
        if (lane == kWave - 1) base = atomicAdd(&sh_count[parity], incl);
        base = lane63(base);
        int pos = base + incl - cnt;
        while (keep) {
            const int bit = __ffs((int)keep) - 1;
            keep &= keep - 1;
            sh_queue[pos++] = (uint16_t)(i0 + bit - c0);
        }
        __syncthreads();
        const int n = sh_count[parity];
        if (threadIdx.x == 0) sh_count[parity ^ 1] = 0;  // the next chunk's counter
        // (3) search the queued draws, up to kSlots per thread at a time (a
        // chunk's share of one part is about kQueue / kParts = 2 per thread;
        // the third slot keeps the usual overshoot in the same pass). The
        // trip count is the same for every thread: the line count is a
        // wave-wide operation.
        for (int it = 0; it < n; it += kSlots * kSearchThreads) {
            const int idx = it + (int)threadIdx.x;
            int64_t i[kSlots], j[kSlots], gbase[kSlots], len[kSlots];
            bool on[kSlots];
            double x[kSlots];
#pragma unroll
            for (int k = 0; k < kSlots; ++k) {
                const int at = idx + k * kSearchThreads;
                on[k] = at < n;
                i[k] = on[k] ? c0 + sh_queue[at] : 0;
                x[k] = multinomial_draw(seed, instance, i[k], W, capW);
                const int b = bk.of(x[k]);
                const int glo = sh_guide[b], ghi = sh_guide[b + 1];
                const int g = glo + first_above_lds(sh_sub + glo, ghi - glo + 1, x[k]);
                gbase[k] = start + (int64_t)g * S;
                len[k] = min(S, end - gbase[k]);
            }
            // Groups wider than one 128-byte line (S > 16, beyond 2^20
            // particles): narrow each draw to the line holding its ancestor,
            // the first line whose last C' exceeds x, by bisecting the line
            // ends (the group's last line ends at the group's end, above x,
            // and is never read). The slots step together, so their loads
            // overlap.
            if (WIDE) {
                int64_t lbase[kSlots];
#pragma unroll
                for (int k = 0; k < kSlots; ++k) lbase[k] = 0;
                for (int64_t span = S / 16; span > 1;) {
                    const int64_t half = span >> 1;
#pragma unroll
                    for (int k = 0; k < kSlots; ++k) {
                        const int64_t q = lbase[k] + half - 1;  // the line end probed
                        const int64_t e = gbase[k] + 16 * q + 15;
                        if (16 * q + 16 < len[k] && C[e] <= x[k]) lbase[k] += half;
                    }
                    span -= half;
                }
#pragma unroll
                for (int k = 0; k < kSlots; ++k) {
                    gbase[k] += 16 * lbase[k];
                    len[k] = min((int64_t)16, len[k] - 16 * lbase[k]);
                }
            }
#pragma unroll
            for (int k = 0; k < kSlots; ++k) {
                if (__ballot(on[k]) == 0) continue;  // wave-uniform
                const bool coop = on[k] && vec && len[k] == 16;
                const int cnt = vec ? line_count_coop(C, x[k], gbase[k], coop,
                                                      sh_xw + kWave * wave_id(),
                                                      sh_gw + kWave * wave_id())
                                    : 0;
                if (on[k])
                    j[k] = coop ? gbase[k] + cnt
                                : gbase[k] + first_above(C + gbase[k], len[k], x[k]);
            }
#pragma unroll
            for (int k = 0; k < kSlots; ++k) {
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

// Multinomial for at most kSmallMultiTiles tiles in one block and one launch:
// the tile sums, the boundaries and each tile's C' come from the same
// functions, in the same order, as in the tile, table and cumulative launches
// (so the same bits), kept in LDS; then each thread bisects C' for eight
// draws at a time. At these sizes the four dependent launches of the general
// path cost more than the whole resampling.
constexpr int64_t kSmallMultiTiles = 2;  // one block runs the tiles one after another
static_assert(kSmallMultiTiles * kTile >= 16, "the search's line count may read C[0..15]");
constexpr int kSmallDraws = 8;           // draws per thread per pass

__global__ __launch_bounds__(kTileThreads) void multinomial_small_kernel(
    const float *__restrict__ lw, int32_t *__restrict__ anc, int64_t P, uint64_t seed,
    uint32_t instance, double *C, char *ws_raw, int32_t *status, Rows rows)
{
    __shared__ double sh_C[kSmallMultiTiles * kTile];
    __shared__ double sh_bound[kSmallMultiTiles];
    const WsView ws = ws_view(ws_raw, P);
    const int64_t n = num_tiles(P);
    for (int64_t t = 0; t < n; ++t) tile_reduce_body(lw, P, t, ws_raw);
    __threadfence_block();
    __syncthreads();
    const TableSums sums = boundaries<false>(ws, P, sh_bound);
    if (threadIdx.x == 0) {
        WsHeader *h = ws.h;
        h->flags = sums.flags;
        h->m = sums.m;
        h->W = sums.W;
        h->delta = sums.W / (double)P;
        h->lse = sums.flags ? ((sums.flags & (kFlagNan | kFlagPosInf)) ? (double)NAN
                                                                       : -(double)INFINITY)
                            : (double)sums.m + log(sums.W);
        if (sums.flags) raise_flags(status, sums.flags);
    }
    if (sums.flags) {  // flagged input: identity ancestors and rows
        for (int64_t i = threadIdx.x; i < P; i += kTileThreads) {
            anc[i] = (int32_t)i;
            C[i] = (double)NAN;
            if (rows.x_in) copy_row(rows, i, i, 0, 1);
        }
        return;
    }
    for (int64_t t = 0; t < n; ++t) {
        float v[4];
        load_tile4(lw, P, t, v);
        double w[4], Cv[4];
        tile_weights(v, sums.m, w);
        tile_cumulative(w, t > 0 ? sh_bound[t - 1] : 0.0, sh_bound[t], sh_C + t * kTile, Cv);
        store_cumw(C, P, t, Cv);
    }
    // a_i = first j with C'_j > x_i; C'_{P-1} = W exceeds every draw
    const double W = sums.W, capW = below(W);
    const int np = (int)P;
    for (int i0 = 0; i0 < np; i0 += kSmallDraws * kTileThreads) {
        double x[kSmallDraws];
        int j[kSmallDraws];
#pragma unroll
        for (int k = 0; k < kSmallDraws; ++k) {
            const int i = i0 + k * kTileThreads + (int)threadIdx.x;
            x[k] = multinomial_draw(seed, instance, i < np ? i : 0, W, capW);
            j[k] = 0;
        }
        for (int len = np; len > 1;) {  // the bisection of first_above_lds, eight at a time
            const int half = len >> 1;
#pragma unroll
            for (int k = 0; k < kSmallDraws; ++k)
                j[k] = sh_C[j[k] + half - 1] <= x[k] ? j[k] + half : j[k];
            len -= half;
        }
#pragma unroll
        for (int k = 0; k < kSmallDraws; ++k) {
            const int i = i0 + k * kTileThreads + (int)threadIdx.x;
            if (i < np) {
                anc[i] = j[k];
                if (rows.x_in) copy_row(rows, i, j[k], 0, 1);
            }
        }
    }
}

}  // namespace

// ---------------------------------------------------------------- launchers
namespace {
std::atomic<int> g_prefix_path{kPathAuto};
std::atomic<int64_t> g_onepass_wait_ns{-1};
constexpr int64_t kOnePassWaitNs = 100000;  // bound of a block's wait for the others' tiles

struct OnePassDevice {
    int64_t capacity[3] = {-1, -1, -1};  // co-resident blocks per row width (0, 1-2, 4)
    int64_t ticks_per_ms = 0;            // real-time clock
};
std::mutex g_onepass_mutex;
OnePassDevice g_onepass_dev[64];

template <int KIND, int DS>
const void *onepass_fn()
{
    return reinterpret_cast<const void *>(&onepass_kernel<KIND, DS>);
}

size_t onepass_smem(int DS) { return (size_t)kOnePassTiles * kTile * DS * sizeof(float); }

// Blocks of onepass_kernel<KIND, DS> the device holds at once, and the
// real-time clock rate; 0 capacity: unknown (the caller uses the launches).
int onepass_device(const void *fn, int slot, size_t smem, int64_t *capacity, int64_t *ticks_per_ms)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return record_hip_error(e);
    if (dev < 0 || dev >= 64) {
        *capacity = 0;
        return 0;
    }
    std::lock_guard<std::mutex> lock(g_onepass_mutex);
    OnePassDevice &d = g_onepass_dev[dev];
    if (d.capacity[slot] < 0) {
        int per_cu = 0, cus = 0, khz = 0;
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kTileThreads, smem);
        if (e != hipSuccess) return record_hip_error(e);
        e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e != hipSuccess) return record_hip_error(e);
        e = hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev);
        if (e != hipSuccess) return record_hip_error(e);
        d.capacity[slot] = (int64_t)per_cu * cus;
        d.ticks_per_ms = khz;
    }
    *capacity = d.capacity[slot];
    *ticks_per_ms = d.ticks_per_ms;
    return 0;
}

// Launches the one-pass stratified/systematic kernel when the call qualifies
// (at most kOnePassMaxTiles tiles, enough co-resident blocks, the path
// setting allows it). *done = false: the caller runs the launches instead.
template <int KIND>
int try_onepass(const float *lw, int32_t *anc, int32_t *off, int64_t P, uint64_t seed,
                uint32_t instance, double *cumw, char *w, int32_t *status, hipStream_t stream,
                const Rows &rows, bool *done)
{
    *done = false;
    const int path = g_prefix_path.load();
    const int64_t n = num_tiles(P);
    if (path != kPathOnePass || n > kOnePassMaxTiles) return 0;  // auto: the launches (faster)
    const int64_t G = (n + kOnePassTiles - 1) / kOnePassTiles;
    if (num_windows(P) > (int64_t)kOnePassWindows * G) return 0;
    const bool staged = rows.x_in && (rows.D == 1 || rows.D == 2 || rows.D == 4) &&
                        (((uintptr_t)rows.x_in) & 15) == 0;
    const int DS = staged ? rows.D : 0;
    const void *fn;
    int slot;
    if (DS == 0) fn = onepass_fn<KIND, 0>(), slot = 0;
    else if (DS == 1) fn = onepass_fn<KIND, 1>(), slot = 1;
    else if (DS == 2) fn = onepass_fn<KIND, 2>(), slot = 1;
    else fn = onepass_fn<KIND, 4>(), slot = 2;
    const size_t smem = onepass_smem(DS);
    int64_t capacity = 0, ticks_per_ms = 0;
    if (const int rc = onepass_device(fn, slot, smem, &capacity, &ticks_per_ms)) return rc;
    if (G > capacity) return 0;
    const int64_t wait_ns = g_onepass_wait_ns.load() < 0 ? kOnePassWaitNs : g_onepass_wait_ns.load();
    const uint64_t ticks = (uint64_t)(wait_ns * ticks_per_ms / 1000000);
    if (smem && allow_dynamic_lds(fn, smem)) return -3;
    // the published words start at zero, which no published word equals
    if (const int rc = launch_zero(w + ws_layout(P, false).pub, (size_t)n * 3 * sizeof(uint64_t),
                                   stream))
        return rc;
    const dim3 grid((uint32_t)G), tb(kTileThreads);
    switch (DS) {
    case 0:
        hipLaunchKernelGGL((onepass_kernel<KIND, 0>), grid, tb, smem, stream, lw, anc, off, P, seed,
                           instance, cumw, w, status, rows, ticks);
        break;
    case 1:
        hipLaunchKernelGGL((onepass_kernel<KIND, 1>), grid, tb, smem, stream, lw, anc, off, P, seed,
                           instance, cumw, w, status, rows, ticks);
        break;
    case 2:
        hipLaunchKernelGGL((onepass_kernel<KIND, 2>), grid, tb, smem, stream, lw, anc, off, P, seed,
                           instance, cumw, w, status, rows, ticks);
        break;
    default:
        hipLaunchKernelGGL((onepass_kernel<KIND, 4>), grid, tb, smem, stream, lw, anc, off, P, seed,
                           instance, cumw, w, status, rows, ticks);
        break;
    }
    *done = true;
    return 0;
}
}  // namespace

int set_prefix_path(int path, int64_t wait_ns)
{
    if (path != kPathAuto && path != kPathLaunches && path != kPathOnePass) return -1;
    g_prefix_path.store(path);
    g_onepass_wait_ns.store(wait_ns < 0 ? -1 : wait_ns);
    return 0;
}

int get_prefix_path() { return g_prefix_path.load(); }

int launch_prefix(int kind, const float *lw, int32_t *anc, int32_t *off, int64_t P, uint64_t seed,
                  uint32_t instance, double *cumw, void *ws, int32_t *status,
                  hipStream_t stream, const Rows &rows)
{
    const int64_t n = num_tiles(P);
    char *w = static_cast<char *>(ws);
    const dim3 tb(kTileThreads);
    if (kind == kMultinomial && n <= kSmallMultiTiles) {
        double *C = cumw ? cumw : reinterpret_cast<double *>(w + ws_layout(P, true).cumw);
        hipLaunchKernelGGL(multinomial_small_kernel, dim3(1), tb, 0, stream, lw, anc, P, seed,
                           instance, C, w, status, rows);
        return launch_status();
    }
    if (kind == kStratified || kind == kSystematic) {
        bool done = false;
        const int rc = kind == kStratified
                           ? try_onepass<kStratified>(lw, anc, off, P, seed, instance, cumw, w,
                                                      status, stream, rows, &done)
                           : try_onepass<kSystematic>(lw, anc, off, P, seed, instance, cumw, w,
                                                      status, stream, rows, &done);
        if (rc) return rc;
        if (done) return launch_status();
    }
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
        if (n <= kFusedCumulativeTiles) {
            hipLaunchKernelGGL(cumulative_kernel<true>, dim3((uint32_t)n), tb, 0, stream, lw, P, C,
                               w, seed, instance, status);
        } else {
            if (const int rc = launch_table<kMultinomial>(P, seed, instance, w, status, nullptr,
                                                          stream))
                return rc;
            hipLaunchKernelGGL(cumulative_kernel<false>, dim3((uint32_t)n), tb, 0, stream, lw, P,
                               C, w, seed, instance, status);
        }
        const size_t smem = (size_t)sub_per_part(P) * sizeof(double);
        const bool wide = sub_stride(P) > 16;
        const void *search = wide ? reinterpret_cast<const void *>(&multinomial_search_kernel<true>)
                                  : reinterpret_cast<const void *>(&multinomial_search_kernel<false>);
        if (allow_dynamic_lds(search, smem)) return -3;
        // K blocks per part: one per CU of an XCD at most, and 16384 draws
        // each at least (a block's range is then one chunk up to 2^20)
        int64_t K = (P + 16383) / 16384;
        K = K < 1 ? 1 : (K > 32 ? 32 : K);
        const int64_t grid = kParts * K;
        if (wide)
            hipLaunchKernelGGL(multinomial_search_kernel<true>, dim3((uint32_t)grid),
                               dim3(kSearchThreads), smem, stream, C, anc, P, seed, instance, w,
                               rows);
        else
            hipLaunchKernelGGL(multinomial_search_kernel<false>, dim3((uint32_t)grid),
                               dim3(kSearchThreads), smem, stream, C, anc, P, seed, instance, w,
                               rows);
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

// Workspace of the no-allocation entry point (resample_prefix_static): a
// file-scope device array, one per GPU the library runs on, held until the
// process ends. In host code `scratch` names a host-side stand-in, not the
// device memory: its device address comes from hipGetSymbolAddress, looked up
// once per device (with that device current) and kept here.
static __device__ __align__(256) char scratch[RS_STATIC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void *g_scratch[kMaxDevices] = {};
}  // namespace

int static_scratch(void **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return record_hip_error(e);
    if (dev < 0 || dev >= kMaxDevices) return -1;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return record_hip_error(e);
        if (!p) return -3;
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return 0;
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
