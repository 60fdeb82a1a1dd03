// Device bodies of the prefix-sum resamplers, shared by the single-call
// kernels (prefix.hip) and the batched persistent kernels (batch.hip) so that
// a resampling instance computes exactly the same values on either path.
// See prefix.hip for the method and the design.
//
// Every body is executed by all kTileThreads threads of a block; decisions
// that lead to a barrier are uniform across the block.
#pragma once

#include <hip/hip_runtime.h>

#include "analysis.h"
#include "common.h"
#include "prefix.h"

namespace rs {
namespace pfx {

constexpr int kNW = kTileThreads / kWave;  // waves per block

// ---------------------------------------------------------------- block ops
__device__ inline double block_sum(double v, double *red)
{
    v = wave_sum(v);
    if (lane_id() == 0) red[wave_id()] = v;
    __syncthreads();
    double s = red[0];
    for (int w = 1; w < kNW; ++w) s += red[w];
    __syncthreads();
    return s;
}

// Exclusive prefix sum over threads.
__device__ inline double block_exclusive_sum(double v, double *red)
{
    const int lane = lane_id(), wave = wave_id();
    const double incl = wave_inclusive_sum(v);
    const double excl = wave_shift_up(incl);
    if (lane == kWave - 1) red[wave] = incl;
    __syncthreads();
    double wp = 0.0;
    for (int w = 0; w < wave; ++w) wp += red[w];
    __syncthreads();
    return wp + excl;
}

// Exclusive prefix maximum over threads of non-negative values (0 first).
__device__ inline double block_exclusive_max(double v, double *red)
{
    const int lane = lane_id(), wave = wave_id();
    const double incl = wave_inclusive_max_nonneg(v);
    const double excl = wave_shift_up(incl);
    if (lane == kWave - 1) red[wave] = incl;
    __syncthreads();
    double wp = 0.0;
    for (int w = 0; w < wave; ++w) wp = fmax(wp, red[w]);
    __syncthreads();
    return fmax(wp, excl);
}

__device__ inline int64_t block_exclusive_isum(int64_t v, int64_t *red, int64_t *total)
{
    const int lane = lane_id(), wave = wave_id();
    const int64_t incl = wave_scan(v, (int64_t)0, AddOp{});
    const int64_t excl = wave_shift_up(incl);
    if (lane == kWave - 1) red[wave] = incl;
    __syncthreads();
    int64_t wp = 0, tot = 0;
    for (int w = 0; w < kNW; ++w) {
        if (w < wave) wp += red[w];
        tot += red[w];
    }
    __syncthreads();
    *total = tot;
    return wp + excl;
}

// The four consecutive log-weights of this thread in tile t (-inf past P).
__device__ __forceinline__ void load_tile4(const float *__restrict__ lw, int64_t P, int64_t t,
                                           float v[4])
{
    const int64_t base = t * kTile + 4 * (int64_t)threadIdx.x;
    const bool aligned = (((uintptr_t)lw) & 15) == 0;
    if (aligned && base + 3 < P) {
        const float4 q = *reinterpret_cast<const float4 *>(lw + base);
        v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
    } else {
#pragma unroll
        for (int k = 0; k < 4; ++k) v[k] = (base + k < P) ? lw[base + k] : -INFINITY;
    }
}

struct WsView {
    WsHeader *h;
    float *tile_max;
    double *tile_sum;
    int32_t *tile_flags;
    double *bound;
    int32_t *count;
    int32_t *win;
    double *sub;
    uint16_t *guide;
    uint8_t *part;
};

__device__ __forceinline__ WsView ws_view(char *ws, int64_t P)
{
    const WsLayout L = ws_layout(P, false);
    WsView v;
    v.h = reinterpret_cast<WsHeader *>(ws + L.header);
    v.tile_max = reinterpret_cast<float *>(ws + L.tile_max);
    v.tile_sum = reinterpret_cast<double *>(ws + L.tile_sum);
    v.tile_flags = reinterpret_cast<int32_t *>(ws + L.tile_flags);
    v.bound = reinterpret_cast<double *>(ws + L.bound);
    v.count = reinterpret_cast<int32_t *>(ws + L.count);
    v.win = reinterpret_cast<int32_t *>(ws + L.win);
    v.sub = reinterpret_cast<double *>(ws + L.sub);
    v.guide = reinterpret_cast<uint16_t *>(ws + L.guide);
    v.part = reinterpret_cast<uint8_t *>(ws + L.part);
    return v;
}

// ------------------------------------------------------ draw points
template <int KIND>
__device__ __forceinline__ double draw_point(int64_t i, double delta, uint64_t seed,
                                             uint32_t instance, double u_sys)
{
    if (KIND == kStratified) {
        const Block4 b = philox(seed, (uint32_t)(i >> 2), instance, 0u, kTagStratified);
        return ((double)i + unit32(word(b, (uint32_t)(i & 3)))) * delta;
    }
    return ((double)i + u_sys) * delta;
}

__device__ __forceinline__ double systematic_offset(uint64_t seed, uint32_t instance)
{
    return unit32(philox(seed, 0u, instance, 0u, kTagSystematic).r0);
}

// N(c) for c < W by bisection over the draw indices [lo, hi) (N(c) is known
// to lie there): one draw point per step, few registers.
template <int KIND>
__device__ int64_t count_below_bisect(double c, int64_t lo, int64_t hi, double delta,
                                      uint64_t seed, uint32_t instance, double u_sys)
{
    while (lo < hi) {
        const int64_t mid = lo + ((hi - lo) >> 1);
        if (draw_point<KIND>(mid, delta, seed, instance, u_sys) < c) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// N(c) = #{i : x_i < c} for the non-decreasing stratified/systematic draw
// points, or P when c >= W (draws at or past W belong to the last positive
// tile). With e = floor(c / (W/P)), x_{e-2} < c <= x_{e+2} up to rounding, so
// the five draws e-2 .. e+2 (two Philox blocks) settle the answer; a
// bisection over all P covers anything else.
template <int KIND>
__device__ int64_t count_below(double c, int64_t P, double W, double delta, uint64_t seed,
                               uint32_t instance, double u_sys)
{
    if (c >= W) return P;
    if (!(c > 0.0)) return 0;
    const double est = floor(c / delta);
    const int64_t e = est > (double)P ? P : (int64_t)est;
    const int64_t s = e >= 2 ? e - 2 : 0;  // window s .. s+4
    double x[5];
    if (KIND == kStratified) {
        const Block4 b0 = philox(seed, (uint32_t)(s >> 2), instance, 0u, kTagStratified);
        const Block4 b1 = philox(seed, (uint32_t)(s >> 2) + 1u, instance, 0u, kTagStratified);
        const uint32_t r[8] = {b0.r0, b0.r1, b0.r2, b0.r3, b1.r0, b1.r1, b1.r2, b1.r3};
        const int off = (int)(s & 3);
#pragma unroll
        for (int k = 0; k < 5; ++k) x[k] = ((double)(s + k) + unit32(r[off + k])) * delta;
    } else {
#pragma unroll
        for (int k = 0; k < 5; ++k) x[k] = ((double)(s + k) + u_sys) * delta;
    }
    // valid when every draw before the window is below c: s = 0 or x_s < c
    if (s == 0 || x[0] < c) {
#pragma unroll
        for (int k = 0; k < 5; ++k) {
            if (s + k >= P) return P;
            if (x[k] >= c) return s + k;
        }
    }
    return count_below_bisect<KIND>(c, 0, P, delta, seed, instance, u_sys);  // not expected
}

// ------------------------------------------------------ phase 1: tile
// A tile's max, sum of exp(lw - max) in binary64 and data flags from the
// block's four log-weights per thread (every thread gets the results).
__device__ inline void tile_reduce_vals(const float v[4], float *mx_out, double *s_out, int *fl_out)
{
    __shared__ double redd[kNW];
    __shared__ float redf[kNW];
    __shared__ int redi[kNW];
    int fl = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if (isnan(v[k])) fl |= kFlagNan;
        else if (isinf(v[k]) && v[k] > 0.0f) fl |= kFlagPosInf;
    }
    // maximum and flags in one barrier (redf/redi are next written after the
    // barriers of the sum below)
    float mx = wave_max(fmaxf(fmaxf(v[0], v[1]), fmaxf(v[2], v[3])));
    fl = wave_or(fl);
    if (lane_id() == 0) {
        redf[wave_id()] = mx;
        redi[wave_id()] = fl;
    }
    __syncthreads();
    mx = redf[0];
    fl = redi[0];
#pragma unroll
    for (int w = 1; w < kNW; ++w) {
        mx = fmaxf(mx, redf[w]);
        fl |= redi[w];
    }
    double s = 0.0;
    if (mx > -INFINITY) {
#pragma unroll
        for (int k = 0; k < 4; ++k) s += exp((double)v[k] - (double)mx);
    }
    *s_out = block_sum(s, redd);
    *mx_out = mx;
    *fl_out = fl;
}

__device__ inline void tile_reduce_body(const float *__restrict__ lw, int64_t P, int64_t t,
                                        char *ws_raw)
{
    const WsView ws = ws_view(ws_raw, P);
    float v[4];
    load_tile4(lw, P, t, v);
    float mx;
    double s;
    int fl;
    tile_reduce_vals(v, &mx, &s, &fl);
    if (threadIdx.x == 0) {
        ws.tile_max[t] = mx;
        ws.tile_sum[t] = s;
        ws.tile_flags[t] = fl;
    }
}

// ------------------------------------------------------ phase 2: table
// Tile boundaries B_t of all n tiles into bound[] (LDS or the workspace):
// global max, tile sums rescaled to it, an exclusive block scan plus a
// per-thread running sum, then a running maximum so B never decreases. Every
// caller (table kernel, fused fill, batched table) runs exactly this code, so
// the boundaries are the same bits on every path. Returns the data flags
// (then bound is unspecified), the max log-weight m and the total W.
//
// Each thread owns a contiguous run of tiles. Up to kRegTiles per thread
// (n <= 1024) the run lives in registers and all its loads are in flight at
// once; longer runs go through bound[]. Both paths perform the same
// operations in the same order.
struct TableSums {
    int flags;
    float m;
    double W;
};

constexpr int kRegTiles = 4;
constexpr int kRunBatch = 8;  // a thread's run is read this many entries at a time

// 16-byte vector groups (four tiles each) a thread has in flight at once in
// the long-run passes: fewer with wide blocks, whose threads have fewer
// registers and fewer groups each.
template <int NT>
constexpr int load_groups()
{
    return NT >= 1024 ? 2 : 4;
}

// The boundaries once each thread holds its run's tile values: in
// registers (reg: mt, S for tiles t0 .. t1-1, at most kRegTiles) or, for
// longer runs, the sums in bound[] and the maxima in ws.tile_max; fl and m
// are the thread's OR of flags and max over its run. LONG: callers that may
// pass more than 1024 tiles (the table launches), where the element-wise
// passes load 16-byte vectors, load_groups() groups at a time; the other
// callers keep the compact strided loops (same operations on every value,
// so the same bits, with fewer registers). NT: the block's threads (a
// multiple of kTileThreads). The runs and their scans always belong to the
// first kTileThreads threads (tile_run), so the association of every sum is
// the same for any NT; the other threads only share the element-wise passes
// and see empty runs.
template <bool LONG, int NT = kTileThreads>
__device__ __forceinline__ TableSums boundaries_tail(const WsView &ws, int64_t n, int64_t t0, int64_t t1,
                                            bool reg, int fl, float m, float mt[kRegTiles],
                                            double S[kRegTiles], double *bound);

// The thread's run of tiles for boundaries(): [t0, t1), and whether it fits
// in registers.
__device__ __forceinline__ void tile_run(int64_t n, int64_t *t0, int64_t *t1, bool *reg)
{
    int64_t per = (n + kTileThreads - 1) / kTileThreads;
    *reg = per <= kRegTiles;  // uniform
    // Longer runs get an odd length, so that the 64 runs of a wave start in
    // different LDS banks (an even length in doubles puts every lane's k-th
    // element in the same bank).
    if (!*reg) per |= 1;
    *t0 = min(n, (int64_t)threadIdx.x * per);
    *t1 = min(n, *t0 + per);
}

template <bool LONG, int NT = kTileThreads>
__device__ inline TableSums boundaries(const WsView &ws, int64_t P, double *bound)
{
    static_assert(NT % kTileThreads == 0, "whole 256-thread groups");
    const int64_t n = num_tiles(P);
    const int tid = threadIdx.x;
    int64_t t0, t1;
    bool reg;
    tile_run(n, &t0, &t1, &reg);
    int fl = 0;
    float m = -INFINITY;
    float mt[kRegTiles];
    double S[kRegTiles];
    if (reg && t1 - t0 == kRegTiles) {
        // a whole run: 16-byte loads (the sections are 256-byte aligned and
        // t0 is a multiple of kRegTiles here)
        static_assert(kRegTiles == 4, "one float4 of maxima, two double2 of sums");
        const float4 m4 = *reinterpret_cast<const float4 *>(ws.tile_max + t0);
        const double2 s01 = *reinterpret_cast<const double2 *>(ws.tile_sum + t0);
        const double2 s23 = *reinterpret_cast<const double2 *>(ws.tile_sum + t0 + 2);
        const int4 f4 = *reinterpret_cast<const int4 *>(ws.tile_flags + t0);
        mt[0] = m4.x, mt[1] = m4.y, mt[2] = m4.z, mt[3] = m4.w;
        S[0] = s01.x, S[1] = s01.y, S[2] = s23.x, S[3] = s23.y;
        fl = f4.x | f4.y | f4.z | f4.w;
#pragma unroll
        for (int k = 0; k < kRegTiles; ++k) m = fmaxf(m, mt[k]);
    } else if (reg) {
#pragma unroll
        for (int k = 0; k < kRegTiles; ++k) {
            const int64_t t = t0 + k;
            const bool in = t < t1;
            mt[k] = in ? ws.tile_max[t] : -INFINITY;
            S[k] = in ? ws.tile_sum[t] : 0.0;
            fl |= in ? ws.tile_flags[t] : 0;
        }
#pragma unroll
        for (int k = 0; k < kRegTiles; ++k) m = fmaxf(m, mt[k]);
    } else if (LONG) {
        // longer runs: the element-wise passes go block-wide (four
        // consecutive tiles per thread and 16-byte vectors, kLoadGroups
        // groups issued before the first is used; the sections are 256-byte
        // aligned); only the sums below follow each thread's contiguous run.
        // The maximum and the OR do not depend on the order they are taken in.
        constexpr int64_t span = 4 * NT;
        constexpr int kLoadGroups = load_groups<NT>();
        const int64_t n4 = n & ~(int64_t)3;
        for (int64_t c = 4 * (int64_t)tid; c < n4; c += span * kLoadGroups) {
            float4 mv[kLoadGroups];
            int4 fv[kLoadGroups];
            double2 sv[2 * kLoadGroups];
#pragma unroll
            for (int j = 0; j < kLoadGroups; ++j) {
                const int64_t t = c + j * span, tc = t < n4 ? t : 0;  // reads stay in the arrays
                mv[j] = *reinterpret_cast<const float4 *>(ws.tile_max + tc);
                fv[j] = *reinterpret_cast<const int4 *>(ws.tile_flags + tc);
                sv[2 * j] = *reinterpret_cast<const double2 *>(ws.tile_sum + tc);
                sv[2 * j + 1] = *reinterpret_cast<const double2 *>(ws.tile_sum + tc + 2);
            }
#pragma unroll
            for (int j = 0; j < kLoadGroups; ++j) {
                const int64_t t = c + j * span;
                if (t < n4) {
                    fl |= fv[j].x | fv[j].y | fv[j].z | fv[j].w;
                    m = fmaxf(m, fmaxf(fmaxf(mv[j].x, mv[j].y), fmaxf(mv[j].z, mv[j].w)));
                    bound[t] = sv[2 * j].x;
                    bound[t + 1] = sv[2 * j].y;
                    bound[t + 2] = sv[2 * j + 1].x;
                    bound[t + 3] = sv[2 * j + 1].y;
                }
            }
        }
        for (int64_t t = n4 + tid; t < n; t += NT) {
            fl |= ws.tile_flags[t];
            m = fmaxf(m, ws.tile_max[t]);
            bound[t] = ws.tile_sum[t];
        }
    } else {
#pragma unroll 8
        for (int64_t t = tid; t < n; t += NT) {
            fl |= ws.tile_flags[t];
            m = fmaxf(m, ws.tile_max[t]);
            bound[t] = ws.tile_sum[t];
        }
    }
    return boundaries_tail<LONG, NT>(ws, n, t0, t1, reg, fl, m, mt, S, bound);
}

template <bool LONG, int NT>
__device__ __forceinline__ TableSums boundaries_tail(const WsView &ws, int64_t n, int64_t t0, int64_t t1,
                                            bool reg, int fl, float m, float mt[kRegTiles],
                                            double S[kRegTiles], double *bound)
{
    constexpr int NW = NT / kWave;
    __shared__ double redd[NW];
    __shared__ float redf[NW];
    __shared__ int redi[NW];
    __shared__ double sh_W;
    const int tid = threadIdx.x;
    // flags and max in one barrier (redi/redf are next written after later barriers)
    fl = wave_or(fl);
    m = wave_max(m);
    if (lane_id() == 0) {
        redi[wave_id()] = fl;
        redf[wave_id()] = m;
    }
    __syncthreads();
    fl = 0;
    m = -INFINITY;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        fl |= redi[w];
        m = fmaxf(m, redf[w]);
    }
    if (!(m > -INFINITY)) fl |= kFlagAllNegInf;
    if (fl) return TableSums{fl, m, 0.0};
    double local = 0.0;
    if (reg) {
#pragma unroll
        for (int k = 0; k < kRegTiles; ++k) {
            if (t0 + k < t1) {
                S[k] = (mt[k] > -INFINITY) ? S[k] * exp((double)mt[k] - (double)m) : 0.0;
                local += S[k];
            }
        }
    } else {
        const auto rescale = [&](int64_t t, float mc) {
            bound[t] = (mc > -INFINITY) ? bound[t] * exp((double)mc - (double)m) : 0.0;
        };
        if (LONG) {
            // the tiles this thread loaded above, their maxima read again
            // (now from L2) as 16-byte vectors, kLoadGroups groups at a time
            constexpr int64_t span = 4 * NT;
            constexpr int kLoadGroups = load_groups<NT>();
            const int64_t n4 = n & ~(int64_t)3;
            for (int64_t c = 4 * (int64_t)tid; c < n4; c += span * kLoadGroups) {
                float4 mv[kLoadGroups];
#pragma unroll
                for (int j = 0; j < kLoadGroups; ++j) {
                    const int64_t t = c + j * span;
                    mv[j] = *reinterpret_cast<const float4 *>(ws.tile_max + (t < n4 ? t : 0));
                }
#pragma unroll
                for (int j = 0; j < kLoadGroups; ++j) {
                    const int64_t t = c + j * span;
                    if (t < n4) {
                        rescale(t, mv[j].x);
                        rescale(t + 1, mv[j].y);
                        rescale(t + 2, mv[j].z);
                        rescale(t + 3, mv[j].w);
                    }
                }
            }
            for (int64_t t = n4 + tid; t < n; t += NT) rescale(t, ws.tile_max[t]);
        } else {
#pragma unroll 8
            for (int64_t t = tid; t < n; t += NT) rescale(t, ws.tile_max[t]);
        }
        __syncthreads();  // the runs below cross the element-wise ownership (reg is uniform)
        // Each pass reads a batch of the run at once; entries of a batch past
        // the run's end stand for its last entry (so every access stays in
        // the thread's run and none waits on a branch) and change nothing.
        for (int64_t c = t0; c < t1; c += kRunBatch) {
            const int lim = (int)min((int64_t)kRunBatch, t1 - c);
            const double *src = bound + c;
            double v[kRunBatch];
#pragma unroll
            for (int k = 0; k < kRunBatch; ++k) v[k] = src[k < lim ? k : lim - 1];
#pragma unroll
            for (int k = 0; k < kRunBatch; ++k) local = k < lim ? local + v[k] : local;  // in tile order
        }
    }
    double run = block_exclusive_sum(local, redd);
    double tmax = 0.0;
    if (reg) {
#pragma unroll
        for (int k = 0; k < kRegTiles; ++k) {
            if (t0 + k < t1) {
                run += S[k];
                S[k] = run;
                tmax = run;  // running sums grow within a thread
            }
        }
    } else {
        for (int64_t c = t0; c < t1; c += kRunBatch) {
            const int lim = (int)min((int64_t)kRunBatch, t1 - c);
            double *dst = bound + c;
            double v[kRunBatch];
#pragma unroll
            for (int k = 0; k < kRunBatch; ++k) v[k] = dst[k < lim ? k : lim - 1];
#pragma unroll
            for (int k = 0; k < kRunBatch; ++k) {
                run = k < lim ? run + v[k] : run;
                dst[k < lim ? k : lim - 1] = run;  // past the run: the last entry's value again
            }
        }
        if (t0 < t1) tmax = run;  // running sums grow within a thread
    }
    const double carry = block_exclusive_max(tmax, redd);
    if (reg) {
#pragma unroll
        for (int k = 0; k < kRegTiles; ++k) {
            const int64_t t = t0 + k;
            if (t < t1) {
                const double b = fmax(S[k], carry);
                bound[t] = b;
                if (t == n - 1) sh_W = b;
            }
        }
    } else {
        double last = 0.0;
        for (int64_t c = t0; c < t1; c += kRunBatch) {
            const int lim = (int)min((int64_t)kRunBatch, t1 - c);
            double *dst = bound + c;
            double v[kRunBatch];
#pragma unroll
            for (int k = 0; k < kRunBatch; ++k) v[k] = dst[k < lim ? k : lim - 1];
#pragma unroll
            for (int k = 0; k < kRunBatch; ++k) {
                const double b = fmax(v[k], carry);
                dst[k < lim ? k : lim - 1] = b;
                last = k < lim ? b : last;
            }
        }
        if (t0 < t1 && t1 == n) sh_W = last;
    }
    __syncthreads();
    return TableSums{0, m, sh_W};
}

// The table launch: boundaries, and for stratified/systematic the draw
// counts below every boundary and the owners of the overflow windows, into
// the workspace. `bound` is scratch for n tiles and `count` for the block's
// tiles plus one (LDS when they fit, else the workspace arrays). With
// parts > 1 (LDS boundaries only) the launch has that many blocks: each
// rebuilds all boundaries (the same bits) and counts and publishes its own
// share of the tiles; block 0 writes the header.
//
// Overflow windows: the draws of tile t beyond its fill block's slots,
// [M_t, hi_t) with M_t = (lo_t & ~3) + kChunk, go to the kWindow-wide windows
// they meet. Only the tile holding a window's first draw can reach into it
// (a later tile's remainder starts more than kWindow past its own first
// draw), so that tile writes the window's entry: itself or -1. Every entry
// is written exactly once. Inlined into every kernel, so that the LDS
// boundaries are addressed as LDS: a called body would reach them through
// flat (generic) loads and stores, and would carry the call's registers.
template <int KIND, int NT = kTileThreads>
__device__ __forceinline__ void table_body(int64_t P, uint64_t seed, uint32_t instance, char *ws_raw,
                           int32_t *status, double *lse_out, double *bound, int32_t *count,
                           double eps = 0.0, uint32_t B_max = 0, uint32_t *B_used = nullptr,
                           int part = 0, int parts = 1)
{
    const WsView ws = ws_view(ws_raw, P);
    WsHeader *h = ws.h;
    const int64_t n = num_tiles(P);
    const int tid = threadIdx.x;
    const bool staged = bound != ws.bound;
    const TableSums sums = boundaries<true, NT>(ws, P, bound);
    if (sums.flags) {
        if (tid == 0 && part == 0) {
            h->flags = sums.flags;
            h->lse = (sums.flags & (kFlagNan | kFlagPosInf)) ? (double)NAN : -(double)INFINITY;
            h->B = 0;
            if (B_used) *B_used = 0;
            if (lse_out)
                *lse_out = (sums.flags & (kFlagNan | kFlagPosInf)) ? (double)NAN
                                                                   : -(double)INFINITY;
            raise_flags(status, sums.flags);
        }
        return;
    }
    const int64_t u0 = n * part / parts, u1 = n * (part + 1) / parts;  // this block's tiles
    const double W = sums.W, delta = W / (double)P;
    // The header, by the block's last thread: block 0 gives it at most
    // NT - 1 counts, so its log (and eq. (5)'s count) overlap the others'
    // counts instead of following them.
    if (tid == NT - 1 && part == 0) {
        const double lse = (double)sums.m + log(W);
        h->m = sums.m;
        h->W = W;
        h->delta = delta;
        h->lse = lse;
        h->flags = 0;
        if (lse_out) *lse_out = lse;
        if (KIND == kAdaptiveB) {
            // with m the largest log-weight the largest normalised weight is 1 / W
            const uint32_t Bn = iterations_for(P, 1.0 / W, eps);
            const uint32_t B = Bn < B_max ? Bn : B_max;
            h->B = B;
            if (B_used) *B_used = B;
        }
    }
    if (staged)
        for (int64_t t = u0 + tid; t < u1; t += NT) ws.bound[t] = bound[t];
    if (KIND == kStratified || KIND == kSystematic) {
        const double u_sys = KIND == kSystematic ? systematic_offset(seed, instance) : 0.0;
        // counts of tiles [c0, u1), c0 = u0 - 1 (that one gives the first tile's lo);
        // count[t - c0] holds tile t's (the block's own slice of scratch)
        const int64_t c0 = u0 > 0 ? u0 - 1 : 0;
        for (int64_t t = c0 + tid; t < u1; t += NT) {
            const int32_t c = (int32_t)count_below<KIND>(bound[t], P, W, delta, seed, instance, u_sys);
            count[t - c0] = c;
            if (count != ws.count && t >= u0) ws.count[t] = c;
        }
        __syncthreads();
        for (int64_t t = u0 + tid; t < u1; t += NT) {
            const int64_t lo = t > 0 ? count[t - 1 - c0] : 0, hi = count[t - c0];
            const int64_t M = (lo & ~(int64_t)3) + kChunk;
            for (int64_t q = (lo + kWindow - 1) / kWindow; q * kWindow < hi; ++q)
                ws.win[q] = (M < hi && M < (q + 1) * kWindow) ? (int32_t)t : -1;
        }
    }
}

// In-tile cumulative weights C'_j from the thread's four log-weights v:
// C'_j = min(Blo + L_j, Bhi), with L the zero-weight-aware running maximum of
// the tile's scan, and C'_j = Bhi from the tile's last positive weight on.
__device__ __forceinline__ void tile_weights(const float v[4], float m, double w[4])
{
#pragma unroll
    for (int k = 0; k < 4; ++k) w[k] = exp((double)v[k] - (double)m);
}

// w: the thread's four weights exp(lw - m) (tile_weights), computed early by
// callers that can overlap them with other waits.
__device__ inline void tile_cumulative(const double w[4], double Blo, double Bhi, double *Cs,
                                       double Cout[4])
{
    __shared__ double red[kNW];
    __shared__ double sh_total;
    double L[4];
    L[0] = w[0];
    L[1] = L[0] + w[1];
    L[2] = L[1] + w[2];
    L[3] = L[2] + w[3];
    const double prefix = block_exclusive_sum(L[3], red);
    double V[4];
    double run = 0.0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if (w[k] > 0.0) run = prefix + L[k];  // a zero weight repeats its predecessor
        V[k] = run;
    }
    const double carry = block_exclusive_max(run, red);
#pragma unroll
    for (int k = 0; k < 4; ++k) V[k] = fmax(V[k], carry);
    if (threadIdx.x == kTileThreads - 1) sh_total = V[3];
    __syncthreads();
    const double Ltot = sh_total;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const double C = (V[k] == Ltot) ? Bhi : fmin(Blo + V[k], Bhi);
        Cout[k] = C;
        Cs[4 * threadIdx.x + k] = C;
    }
    __syncthreads();
}

// First index j of the kTile-entry Cs with Cs[j] > x (Cs is non-decreasing).
__device__ __forceinline__ int search_tile(const double *Cs, double x)
{
    int j = 0;
#pragma unroll
    for (int step = kTile / 2; step >= 1; step >>= 1)
        if (Cs[j + step - 1] <= x) j += step;
    return j;
}

__device__ __forceinline__ void store_cumw(double *cumw, int64_t P, int64_t t, const double C[4])
{
    const int64_t base = t * kTile + 4 * (int64_t)threadIdx.x;
#pragma unroll
    for (int k = 0; k < 4; ++k)
        if (base + k < P) cumw[base + k] = C[k];
}

// Rows x_out[o, :] = x_in[a_o, :] for o in [ob, oe), a_o = sh_anc[o - a0],
// copied by the whole block (coalesced 16-byte vectors when possible).
__device__ inline void copy_rows_from_lds(const int32_t *sh_anc, int64_t a0, int64_t ob,
                                          int64_t oe, const float *__restrict__ x_in,
                                          float *__restrict__ x_out, int32_t D, int64_t P,
                                          int *fl)
{
    const bool vec = (D % 4 == 0) && ((((uintptr_t)x_in) | ((uintptr_t)x_out)) & 15) == 0;
    if (vec) {
        const int cols = D / 4;
        const int64_t total = (oe - ob) * cols;
        for (int64_t e = threadIdx.x; e < total; e += kTileThreads) {
            const int64_t r = e / cols, c = e - r * cols;
            const int64_t o = ob + r;
            const int32_t a = sh_anc[o - a0];
            float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
            if (a >= 0 && (int64_t)a < P) v = reinterpret_cast<const float4 *>(x_in)[(int64_t)a * cols + c];
            else *fl |= kFlagBadAncestor;
            reinterpret_cast<float4 *>(x_out)[o * cols + c] = v;
        }
    } else {
        const int64_t total = (oe - ob) * D;
        for (int64_t e = threadIdx.x; e < total; e += kTileThreads) {
            const int64_t r = e / D, d = e - r * D;
            const int64_t o = ob + r;
            const int32_t a = sh_anc[o - a0];
            const bool ok = a >= 0 && (int64_t)a < P;
            x_out[o * D + d] = ok ? x_in[(int64_t)a * D + d] : 0.0f;
            if (!ok) *fl |= kFlagBadAncestor;
        }
    }
}

// As copy_rows_from_lds, with the source rows of tile t (particles
// tile_base .. tile_base + kTile - 1) staged in LDS: x_out[o, :] =
// sh_rows[(a_o - tile_base) D ..]. The fill's ancestors lie in its tile.
__device__ inline void copy_rows_staged(const int32_t *sh_anc, int64_t a0, int64_t ob, int64_t oe,
                                        const float *sh_rows, int64_t tile_base,
                                        float *__restrict__ x_out, int32_t D, int *fl)
{
    const bool vec = (D % 4 == 0) && ((((uintptr_t)x_out) & 15) == 0);
    if (vec) {
        const int cols = D / 4;
        const int64_t total = (oe - ob) * cols;
        for (int64_t e = threadIdx.x; e < total; e += kTileThreads) {
            const int64_t r = e / cols, c = e - r * cols;
            const int64_t o = ob + r;
            const int64_t a = (int64_t)sh_anc[o - a0] - tile_base;
            float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
            if (a >= 0 && a < kTile) v = reinterpret_cast<const float4 *>(sh_rows)[a * cols + c];
            else *fl |= kFlagInternal;
            reinterpret_cast<float4 *>(x_out)[o * cols + c] = v;
        }
    } else {
        const int64_t total = (oe - ob) * D;
        for (int64_t e = threadIdx.x; e < total; e += kTileThreads) {
            const int64_t r = e / D, d = e - r * D;
            const int64_t o = ob + r;
            const int64_t a = (int64_t)sh_anc[o - a0] - tile_base;
            const bool ok = a >= 0 && a < kTile;
            x_out[o * D + d] = ok ? sh_rows[a * D + d] : 0.0f;
            if (!ok) *fl |= kFlagInternal;
        }
    }
}

// ------------------------------------------------------ phase 3: fill
// First tile t with B_t > x, for x < W (bisection over n non-decreasing
// boundaries in LDS).
__device__ __forceinline__ int64_t first_bound_above(const double *bound, int64_t n, double x)
{
    int64_t lo = 0, hi = n - 1;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (bound[mid] > x) hi = mid;
        else lo = mid + 1;
    }
    return lo;
}

// Offspring o_j of the four particles j0 .. j0+3 of tile t, j0 = t kTile + 4 tid
// (Sec. 2: o_j is the number of draws whose ancestor is j). When the block
// holds every draw of the tile, [lo, hi), in sh_anc (sorted, slot r = draw
// a0 + r), each run of equal ancestors marks its first slot and its end, and
// o_j is the width of j's run (0 without one); otherwise (a tile whose draws
// spill into overflow windows) o_j = N(C'_j) - N(C'_{j-1}) with N the draw
// count below a point, C'_{-1} = B_{t-1} and N(B_{t-1}) = lo. Both give the
// exact counts of the ancestors the fill writes. Called by the whole block,
// after a barrier that follows the searches: the run marks of the first form
// reuse the LDS of Cs, which that form no longer reads.
template <int KIND>
__device__ void tile_offspring(int32_t *off, int64_t P, int64_t t, int64_t lo, int64_t hi,
                               int64_t oe, int64_t a0, const int32_t a[8],
                               const int32_t *sh_anc, double *Cs, double W, double delta,
                               uint64_t seed, uint32_t instance, double u_sys)
{
    static_assert(2 * kTile * sizeof(int16_t) <= kTile * sizeof(double), "marks fit in Cs");
    int16_t *const sh_start = reinterpret_cast<int16_t *>(Cs), *const sh_stop = sh_start + kTile;
    const int64_t base = t * kTile;
    const int64_t j0 = base + 4 * (int64_t)threadIdx.x;
    int32_t o[4];
    if (hi == oe) {  // uniform: every draw of the tile is in sh_anc
        const int r0 = (int)(lo - a0), r1 = (int)(hi - a0);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            sh_start[4 * threadIdx.x + k] = 0;
            sh_stop[4 * threadIdx.x + k] = 0;
        }
        __syncthreads();
        // the thread's own slots are in registers; only the neighbours across
        // thread boundaries come from LDS
        const int rb = 8 * (int)threadIdx.x;
        const int32_t before = (rb > r0 && rb < r1) ? sh_anc[rb - 1] : -1;
        const int32_t after = (rb + 7 >= r0 && rb + 7 < r1 - 1) ? sh_anc[rb + 8] : -1;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int r = rb + k;
            if (r >= r0 && r < r1) {
                const int32_t ak = a[k];
                const int32_t prev = k == 0 ? before : a[k - 1];
                const int32_t next = k == 7 ? after : a[k + 1];
                const int q = (int)(ak - base);
                if (r == r0 || prev != ak) sh_start[q] = (int16_t)r;
                if (r == r1 - 1 || next != ak) sh_stop[q] = (int16_t)(r + 1);
            }
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < 4; ++k)
            o[k] = (int32_t)sh_stop[4 * threadIdx.x + k] - (int32_t)sh_start[4 * threadIdx.x + k];
    } else {
        if (j0 >= P) return;
        // rare (heavy tiles only): bisection over the tile's draws [lo, hi), one
        // count at a time, which keeps the kernel's registers low; C'_j = B_t
        // (the tile's end) counts hi, also when hi = P takes draws at or past W
        int64_t prev = lo;
#pragma unroll 1
        for (int k = -1; k < 4; ++k) {
            const int e = 4 * (int)threadIdx.x + k;
            int64_t c = lo;
            if (e >= 0)
                c = Cs[e] >= Cs[kTile - 1] ? hi
                                           : count_below_bisect<KIND>(Cs[e], lo, hi, delta, seed,
                                                                      instance, u_sys);
            if (k >= 0) o[k] = (int32_t)(c - prev);
            prev = c;
        }
    }
    if (j0 >= P) return;
    if (j0 + 3 < P && (((uintptr_t)off) & 15) == 0) {
        *reinterpret_cast<int4 *>(off + j0) = make_int4(o[0], o[1], o[2], o[3]);
    } else {
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (j0 + k < P) off[j0 + k] = o[k];
    }
}

// The fill proper, shared by the fill launch and the one-pass launch: the
// block's draw slots [ob, oe) of tile t (slot base a0; the tile's draws are
// [lo, hi), its boundaries Blo and Bhi, wts the thread's four weights
// exp(lw - m)): the tile's cumulative weights in Cs (stored to cumw by a
// tile block), the ancestors of the slots, the tile's offspring (tile block)
// and the rows (from sh_rows, the tile's kTile rows staged in LDS, when given).
template <int KIND>
__device__ __forceinline__ void fill_chunk(int32_t *__restrict__ anc, int32_t *__restrict__ off, int64_t P,
                           uint64_t seed, uint32_t instance, double *cumw, bool tile_block,
                           int64_t t, int64_t ob, int64_t oe, int64_t a0, int64_t lo, int64_t hi,
                           double Blo, double Bhi, double W, const double wts[4],
                           const float *x_in, float *x_out, int32_t D, int32_t *status,
                           double *Cs, int32_t *sh_anc, const float *sh_rows)
{
    const double delta = W / (double)P;
    const double u_sys = KIND == kSystematic ? systematic_offset(seed, instance) : 0.0;
    const bool want_off = off && tile_block;
    double C[4];
    tile_cumulative(wts, Blo, Bhi, Cs, C);  // ends with a barrier
    if (cumw && tile_block) store_cumw(cumw, P, t, C);

    const bool keep = x_in || want_off;  // ancestors needed again from LDS
    const int64_t o0 = a0 + 8 * (int64_t)threadIdx.x;
    int32_t a[8];  // this thread's slots' ancestors (defined for the slots in [ob, oe))
    if (o0 + 8 > ob && o0 < oe) {
        double U[8];
        if (KIND == kStratified) {
            const Block4 b0 = philox(seed, (uint32_t)(o0 >> 2), instance, 0u, kTagStratified);
            const Block4 b1 = philox(seed, (uint32_t)(o0 >> 2) + 1u, instance, 0u, kTagStratified);
            U[0] = unit32(b0.r0); U[1] = unit32(b0.r1); U[2] = unit32(b0.r2); U[3] = unit32(b0.r3);
            U[4] = unit32(b1.r0); U[5] = unit32(b1.r1); U[6] = unit32(b1.r2); U[7] = unit32(b1.r3);
        } else {
#pragma unroll
            for (int k = 0; k < 8; ++k) U[k] = u_sys;
        }
        const double cap = below(Bhi);
        double x[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) x[k] = fmin(((double)(o0 + k) + U[k]) * delta, cap);
        // the draws are non-decreasing, so a_0 <= a_k <= a_7: bisect the whole
        // tile for the first and last draw only, and the six between within
        // [a_0, a_7] (usually a few particles), all six in lockstep; the same
        // first-above rule, so the same ancestors as eight full bisections
        const int32_t tile_base = (int32_t)(t * kTile);
        const int j0 = search_tile(Cs, x[0]), j7 = search_tile(Cs, x[7]);
        int jm[6];
#pragma unroll
        for (int k = 0; k < 6; ++k) jm[k] = j0;
        for (int len = j7 - j0 + 1; len > 1;) {
            const int half = len >> 1;
#pragma unroll
            for (int k = 0; k < 6; ++k) jm[k] = Cs[jm[k] + half - 1] <= x[k + 1] ? jm[k] + half : jm[k];
            len -= half;
        }
        a[0] = tile_base + j0;
        a[7] = tile_base + j7;
#pragma unroll
        for (int k = 0; k < 6; ++k) a[k + 1] = tile_base + jm[k];
        if (anc) {
            const bool full = (o0 >= ob) && (o0 + 8 <= oe) && ((((uintptr_t)(anc + o0)) & 15) == 0);
            if (full) {
                int4 *dst = reinterpret_cast<int4 *>(anc + o0);
                dst[0] = make_int4(a[0], a[1], a[2], a[3]);
                dst[1] = make_int4(a[4], a[5], a[6], a[7]);
            } else {
#pragma unroll
                for (int k = 0; k < 8; ++k)
                    if (o0 + k >= ob && o0 + k < oe) anc[o0 + k] = a[k];
            }
        }
        if (keep) {
#pragma unroll
            for (int k = 0; k < 8; ++k) sh_anc[8 * threadIdx.x + k] = a[k];
        }
    }
    if (keep) __syncthreads();
    if (want_off)
        tile_offspring<KIND>(off, P, t, lo, hi, oe, a0, a, sh_anc, Cs, W,
                             delta, seed, instance, u_sys);
    if (x_in) {
        int fl = 0;
        if (sh_rows) copy_rows_staged(sh_anc, a0, ob, oe, sh_rows, t * kTile, x_out, D, &fl);
        else copy_rows_from_lds(sh_anc, a0, ob, oe, x_in, x_out, D, P, &fl);
        raise_flags(status, fl);
    }
}

// Fill block g of an instance. Block g < n serves tile g's draws [lo, hi)
// as far as its kChunk slots (base lo & ~3) reach, which is all of them
// unless the tile is heavy (more than kChunk - 3 draws); block n + q serves
// the draws of window [q kWindow, (q+1) kWindow) that belong to a heavy
// tile's remainder. Together they cover every draw once.
// With FUSED the block rebuilds the boundaries in LDS (sh_bound, n doubles)
// and counts the draws itself; otherwise it reads the table launch's output.
// Writes the ancestors (anc, may be null), the offspring of the tile (off,
// may be null; tile blocks only) and, with x_in, copies the rows.
// Cs: kTile doubles, sh_anc: kChunk ints of LDS.
template <int KIND, bool FUSED>
__device__ void fill_body(const float *__restrict__ lw, int32_t *__restrict__ anc,
                          int32_t *__restrict__ off, int64_t P, uint64_t seed, uint32_t instance,
                          double *cumw, char *ws_raw, int64_t g, const float *x_in, float *x_out,
                          int32_t D, int32_t *status, double *Cs, int32_t *sh_anc,
                          double *sh_bound)
{
    __shared__ int64_t sh_range[6];  // tile, first draw, end draw, slot base, lo, hi
    __shared__ double sh_b[2];       // B_{t-1}, B_t
    const WsView ws = ws_view(ws_raw, P);
    const int64_t n = num_tiles(P);
    const bool tile_block = g < n;
    float v[4];
    if (tile_block) load_tile4(lw, P, g, v);  // issued before the table reads

    // Table path: thread 0 fetches its table entries before the flags are
    // known (the tile index is clamped, so the speculative reads stay inside
    // the workspace; the values are used only when the flags are clear).
    int64_t s_t = 0, s_lo = 0, s_hi = 0;
    double s_blo = 0.0, s_bhi = 0.0;
    if (!FUSED && threadIdx.x == 0) {
        const int64_t t = tile_block ? g : (int64_t)ws.win[g - n];  // -1: no owner
        const int64_t tc = t < 0 ? 0 : (t >= n ? n - 1 : t);
        s_t = t;
        s_lo = tc > 0 ? ws.count[tc - 1] : 0;
        s_hi = ws.count[tc];
        s_blo = tc > 0 ? ws.bound[tc - 1] : 0.0;
        s_bhi = ws.bound[tc];
    }

    int flags;
    float m;
    double W;
    if (FUSED) {
        const TableSums sums = boundaries<false>(ws, P, sh_bound);
        flags = sums.flags;
        m = sums.m;
        W = sums.W;
        if (g == 0 && threadIdx.x == 0) {
            // the header as the table launch leaves it, for launches that follow
            WsHeader *h = ws.h;
            h->flags = flags;
            h->m = m;
            h->W = W;
            h->delta = W / (double)P;
            h->lse = flags ? ((flags & (kFlagNan | kFlagPosInf)) ? (double)NAN : -(double)INFINITY)
                           : (double)m + log(W);
            if (flags) raise_flags(status, flags);
        }
    } else {
        flags = ws.h->flags;
        m = ws.h->m;
        W = ws.h->W;
    }
    if (flags) {  // flagged input: identity ancestors and rows, one offspring each
        if (tile_block) {
            for (int64_t j = g * kTile + threadIdx.x; j < min(P, (g + 1) * kTile); j += kTileThreads) {
                if (anc) anc[j] = (int32_t)j;
                if (off) off[j] = 1;
                if (cumw) cumw[j] = (double)NAN;
                if (x_in)
                    for (int d = 0; d < D; ++d) x_out[j * D + d] = x_in[j * D + d];
            }
        }
        return;
    }
    const double delta = W / (double)P;
    const double u_sys = KIND == kSystematic ? systematic_offset(seed, instance) : 0.0;

    // The block's tile t (-1: an overflow window nobody owns) and draws
    // [lo, hi). A tile block takes the draws [lo, min(hi, a0 + kChunk)) in the
    // slots of base a0 = lo & ~3; the rest of a heavy tile, [M, hi) with
    // M = a0 + kChunk, goes to the overflow blocks of the windows it meets.
    int64_t t = -1, lo = 0, hi = 0;
    double Blo = 0.0, Bhi = 0.0;
    if (FUSED) {
        // The owner of overflow window q can only be the tile holding its first
        // draw: a tile starting later in the window has its remainder beyond it.
        __shared__ int64_t sh_t, sh_hi;
        if (threadIdx.x == 0) {
            int64_t tt = g;
            if (!tile_block) {
                const double x0 = draw_point<KIND>((g - n) * kWindow, delta, seed, instance, u_sys);
                tt = first_bound_above(sh_bound, n, fmin(x0, below(W)));
            }
            sh_t = tt;
        }
        __syncthreads();
        const int64_t tt = sh_t;
        if (threadIdx.x == kWave)  // the upper count on another wave, in parallel
            sh_hi = count_below<KIND>(sh_bound[tt], P, W, delta, seed, instance, u_sys);
        int64_t lo_t = 0;
        if (threadIdx.x == 0 && tt > 0)
            lo_t = count_below<KIND>(sh_bound[tt - 1], P, W, delta, seed, instance, u_sys);
        __syncthreads();
        if (threadIdx.x == 0) {
            const int64_t hi_t = sh_hi;
            const int64_t q = g - n, M = (lo_t & ~(int64_t)3) + kChunk;
            const bool owner = tile_block || max(q * kWindow, M) < min((q + 1) * kWindow, hi_t);
            if (owner) {
                t = tt;
                lo = lo_t;
                hi = hi_t;
                Blo = tt > 0 ? sh_bound[tt - 1] : 0.0;
                Bhi = sh_bound[tt];
            }
        }
    } else if (threadIdx.x == 0) {
        t = s_t;
        lo = s_lo;
        hi = s_hi;
        Blo = s_blo;
        Bhi = s_bhi;
    }
    // the tile block's weights, while thread 0 settles the range
    double wts[4];
    if (tile_block) tile_weights(v, m, wts);
    if (threadIdx.x == 0) {
        int64_t ob = 0, oe = 0, a0 = 0;
        if (t >= 0) {
            const int64_t base = lo & ~(int64_t)3;
            if (tile_block) {
                a0 = base;
                ob = lo;
                oe = min(hi, base + kChunk);
            } else {
                const int64_t q = g - n;
                ob = max(q * kWindow, base + kChunk);
                oe = min((q + 1) * kWindow, hi);
                a0 = ob & ~(int64_t)3;  // ob - a0 + kWindow <= kChunk
            }
        }
        sh_range[0] = t;
        sh_range[1] = ob;
        sh_range[2] = oe;
        sh_range[3] = a0;
        sh_range[4] = lo;
        sh_range[5] = hi;
        sh_b[0] = Blo;
        sh_b[1] = Bhi;
    }
    __syncthreads();
    t = sh_range[0];
    const int64_t ob = sh_range[1], oe = sh_range[2], a0 = sh_range[3];
    Blo = sh_b[0];
    Bhi = sh_b[1];
    const bool want_off = off && tile_block;
    if (t < 0 || (ob >= oe && !(cumw && tile_block) && !want_off)) return;  // nothing to write
    if (!tile_block) {
        load_tile4(lw, P, t, v);
        tile_weights(v, m, wts);
    }

    fill_chunk<KIND>(anc, off, P, seed, instance, cumw, tile_block, t, ob, oe, a0, sh_range[4],
                     sh_range[5], Blo, Bhi, W, wts, x_in, x_out, D, status, Cs, sh_anc, nullptr);
}

}  // namespace pfx
}  // namespace rs
