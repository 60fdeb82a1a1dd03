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
// Design on MI355X. Launch 1 (tile_reduce_kernel) streams the log-weights once
// and reduces each 1024-weight tile to (max, sum of exp); the block finishing
// last turns the partials into tile boundaries B_t (the cumulative weight at
// each tile end) and a launch table. Launch 2 (fill_kernel) gives each tile
// one 256-thread block (plus extra blocks for tiles that own more than 2048
// outputs): it counts the draw points below its two boundaries, recomputes
// the tile's scan in LDS from a second read of the weights, and merges the
// sorted draw points into it, writing ancestors in order. HBM traffic is the
// algorithmic minimum of two reads of lw and one write of anc; the cumulative
// weights are never stored unless requested. The multinomial resampler's
// draw points are unsorted, so it stores C and searches it (launches 2m, 3m).
//
// Rounding: inside a tile C'_j = min(B_{t-1} + L_j, B_t), where L_j is a
// zero-weight-aware running maximum of the tile's scan, and C'_j = B_t from
// the tile's last positive weight on. This keeps C' non-decreasing across
// tiles although the tile sums and the in-tile scans round differently, and
// keeps zero-weight particles unselectable. C' agrees with the binary64
// sequential sum to a few ulps.
#include <hip/hip_runtime.h>

#include "common.h"
#include "launch.h"
#include "prefix.h"

namespace rs {
namespace {

// ---------------------------------------------------------------- block ops
// All of these are called by every thread of a kTileThreads block.
constexpr int kWaves = kTileThreads / kWave;

__device__ double block_sum(double v, double *red)
{
    v = wave_sum(v);
    if (lane_id() == 0) red[wave_id()] = v;
    __syncthreads();
    double s = red[0];
    for (int w = 1; w < kWaves; ++w) s += red[w];
    __syncthreads();
    return s;
}

__device__ float block_max(float v, float *red)
{
    v = wave_max(v);
    if (lane_id() == 0) red[wave_id()] = v;
    __syncthreads();
    float s = red[0];
    for (int w = 1; w < kWaves; ++w) s = fmaxf(s, red[w]);
    __syncthreads();
    return s;
}

__device__ int block_or(int v, int *red)
{
    v = wave_or(v);
    if (lane_id() == 0) red[wave_id()] = v;
    __syncthreads();
    int s = 0;
    for (int w = 0; w < kWaves; ++w) s |= red[w];
    __syncthreads();
    return s;
}

// Exclusive prefix sum over threads; *total receives the block total.
__device__ double block_exclusive_sum(double v, double *red, double *total)
{
    const int lane = lane_id(), wave = wave_id();
    double incl = wave_inclusive_sum(v);
    double excl = __shfl_up(incl, 1, kWave);
    if (lane == 0) excl = 0.0;
    if (lane == kWave - 1) red[wave] = incl;
    __syncthreads();
    double wp = 0.0;
    for (int w = 0; w < wave; ++w) wp += red[w];
    double tot = red[0];
    for (int w = 1; w < kWaves; ++w) tot += red[w];
    __syncthreads();
    *total = tot;
    return wp + excl;
}

// Exclusive prefix maximum over threads of non-negative values (0 for thread 0).
__device__ double block_exclusive_max(double v, double *red)
{
    const int lane = lane_id(), wave = wave_id();
    double incl = v;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        double y = __shfl_up(incl, off, kWave);
        if (lane >= off) incl = fmax(incl, y);
    }
    double excl = __shfl_up(incl, 1, kWave);
    if (lane == 0) excl = 0.0;
    if (lane == kWave - 1) red[wave] = incl;
    __syncthreads();
    double wp = 0.0;
    for (int w = 0; w < wave; ++w) wp = fmax(wp, red[w]);
    __syncthreads();
    return fmax(wp, excl);
}

__device__ int64_t block_exclusive_isum(int64_t v, int64_t *red, int64_t *total)
{
    const int lane = lane_id(), wave = wave_id();
    int64_t incl = v;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        int64_t y = __shfl_up(incl, off, kWave);
        if (lane >= off) incl += y;
    }
    int64_t excl = __shfl_up(incl, 1, kWave);
    if (lane == 0) excl = 0;
    if (lane == kWave - 1) red[wave] = incl;
    __syncthreads();
    int64_t wp = 0, tot = 0;
    for (int w = 0; w < kWaves; ++w) {
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
    double *bound;
    int32_t *overflow;
    double *cumw;
};

__device__ __forceinline__ WsView ws_view(char *ws, int64_t P, bool with_cumw)
{
    const WsLayout L = ws_layout(P, with_cumw);
    WsView v;
    v.h = reinterpret_cast<WsHeader *>(ws + L.header);
    v.tile_max = reinterpret_cast<float *>(ws + L.tile_max);
    v.tile_sum = reinterpret_cast<double *>(ws + L.tile_sum);
    v.bound = reinterpret_cast<double *>(ws + L.bound);
    v.overflow = reinterpret_cast<int32_t *>(ws + L.overflow);
    v.cumw = with_cumw ? reinterpret_cast<double *>(ws + L.cumw) : nullptr;
    return v;
}

// ------------------------------------------------------ launch 1: tiles
// Last block: global max, scaled tile sums, tile boundaries (inclusive sum,
// then a running maximum so they never decrease), and the fill table.
template <int KIND>
__device__ void build_table(const WsView &ws, int64_t P, int32_t *status, double *lse_out)
{
    __shared__ double redd[kWaves];
    __shared__ float redf[kWaves];
    __shared__ int64_t redi[kWaves];
    __shared__ double sh_W;
    WsHeader *h = ws.h;
    const int64_t n = num_tiles(P);
    const int tid = threadIdx.x;

    int flags = __hip_atomic_load(&h->acc_flags, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    float m = -INFINITY;
    for (int64_t t = tid; t < n; t += kTileThreads) m = fmaxf(m, ws.tile_max[t]);
    m = block_max(m, redf);
    if (!(m > -INFINITY)) flags |= kFlagAllNegInf;
    if (flags) {
        if (tid == 0) {
            h->flags = flags;
            h->acc_flags = 0;
            h->counter = 0;
            if (lse_out)
                *lse_out = (flags & (kFlagNan | kFlagPosInf)) ? (double)NAN : -(double)INFINITY;
            raise_flags(status, flags);
        }
        return;
    }

    // Each thread owns a contiguous run of tiles.
    const int64_t per = (n + kTileThreads - 1) / kTileThreads;
    const int64_t t0 = min(n, (int64_t)tid * per), t1 = min(n, t0 + per);
    double local = 0.0;
    for (int64_t t = t0; t < t1; ++t) {
        const float mt = ws.tile_max[t];
        const double S = (mt > -INFINITY) ? ws.tile_sum[t] * exp((double)mt - (double)m) : 0.0;
        ws.bound[t] = S;  // scaled tile sum, replaced below by the boundary
        local += S;
    }
    double total;
    double run = block_exclusive_sum(local, redd, &total);
    double tmax = 0.0;
    for (int64_t t = t0; t < t1; ++t) {
        run += ws.bound[t];
        ws.bound[t] = run;
        tmax = run;  // inclusive sums grow within a thread
    }
    const double carry = block_exclusive_max(tmax, redd);
    for (int64_t t = t0; t < t1; ++t) {
        const double b = fmax(ws.bound[t], carry);
        ws.bound[t] = b;
        if (t == n - 1) sh_W = b;
    }
    __syncthreads();
    const double W = sh_W;
    const double delta = W / (double)P;

    if (KIND == kStratified || KIND == kSystematic) {
        // Fill blocks per tile: a tile whose weight share is L/delta strata
        // owns at most L/delta + 2 draw points (+3 for 4-aligned chunks).
        int64_t nov = 0;
        for (int64_t t = t0; t < t1; ++t) {
            const double lo = t > 0 ? ws.bound[t - 1] : 0.0;
            const double u = ceil((ws.bound[t] - lo) / delta) + (double)kChunkSlack;
            nov += (int64_t)ceil(u / (double)kChunk) - 1;
        }
        int64_t tot_ov;
        int64_t acc = block_exclusive_isum(nov, redi, &tot_ov);
        for (int64_t t = t0; t < t1; ++t) {
            ws.overflow[t] = (int32_t)acc;
            const double lo = t > 0 ? ws.bound[t - 1] : 0.0;
            const double u = ceil((ws.bound[t] - lo) / delta) + (double)kChunkSlack;
            acc += (int64_t)ceil(u / (double)kChunk) - 1;
        }
        if (tid == 0) {
            ws.overflow[n] = (int32_t)tot_ov;
            h->n_overflow = (int32_t)tot_ov;
        }
    }
    if (tid == 0) {
        h->m = m;
        h->W = W;
        h->delta = delta;
        h->lse = (double)m + log(W);
        h->flags = 0;
        h->acc_flags = 0;
        h->counter = 0;
        if (lse_out) *lse_out = h->lse;
    }
}

// One block per tile: tile max and sum of exp(lw - tile max), data flags;
// the last block to finish builds the table. The header field acc_flags
// accumulates flags across blocks; flags holds the final verdict.
template <int KIND>
__global__ __launch_bounds__(kTileThreads) void tile_reduce_kernel(const float *__restrict__ lw,
                                                                   int64_t P, char *ws_raw,
                                                                   int32_t *status,
                                                                   double *lse_out)
{
    __shared__ double redd[kWaves];
    __shared__ float redf[kWaves];
    __shared__ int redi[kWaves];
    __shared__ int is_last;
    const WsView ws = ws_view(ws_raw, P, false);
    const int64_t n = num_tiles(P);
    const int64_t t = blockIdx.x;

    float v[4];
    load_tile4(lw, P, t, v);
    int fl = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if (isnan(v[k])) fl |= kFlagNan;
        else if (isinf(v[k]) && v[k] > 0.0f) fl |= kFlagPosInf;
    }
    float mx = fmaxf(fmaxf(v[0], v[1]), fmaxf(v[2], v[3]));
    mx = block_max(mx, redf);
    fl = block_or(fl, redi);
    double s = 0.0;
    if (mx > -INFINITY) {
#pragma unroll
        for (int k = 0; k < 4; ++k) s += exp((double)v[k] - (double)mx);
    }
    s = block_sum(s, redd);
    if (threadIdx.x == 0) {
        ws.tile_max[t] = mx;
        ws.tile_sum[t] = s;
        if (fl) atomicOr(&ws.h->acc_flags, fl);
        __threadfence();
        const unsigned prev = atomicAdd(&ws.h->counter, 1u);
        is_last = (prev == (unsigned)(n - 1));
    }
    __syncthreads();
    if (!is_last) return;
    __threadfence();
    build_table<KIND>(ws, P, status, lse_out);
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

// N(c) = #{i : x_i < c} for the non-decreasing stratified/systematic draw
// points, or P when c >= W (the draws at or past W belong to the last
// positive tile). Executed by a whole wave: each round evaluates 64 probes in
// parallel, first around the estimate c / delta, then spread over the
// remaining bracket, so it ends in at most 7 rounds for any P < 2^31.
template <int KIND>
__device__ int64_t count_below(double c, int64_t P, double W, double delta, uint64_t seed,
                               uint32_t instance, double u_sys, int *bad)
{
    if (c >= W) return P;
    if (!(c > 0.0)) return 0;
    const int lane = lane_id();
    int64_t a = 0, b = P;  // answer in [a, b]; x_{a-1} < c and x_b >= c
    double est = floor(c / delta);
    int64_t guess = est < 0.0 ? 0 : (est > (double)P ? P : (int64_t)est);
    for (int round = 0; round < 8; ++round) {
        const int64_t width = b - a;
        int64_t probe;
        if (width <= kWave) {
            probe = a + lane;
            const bool in = lane < width;
            const bool below_c = in && draw_point<KIND>(probe, delta, seed, instance, u_sys) < c;
            const uint64_t mask = __ballot(below_c);
            return a + (int64_t)__popcll(mask);
        }
        if (round == 0) {
            int64_t s = guess - kWave / 2;
            s = s < a ? a : s;
            s = s + kWave > b ? b - kWave : s;
            probe = s + lane;
        } else {
            probe = a + (width * (int64_t)(lane + 1)) / (kWave + 1);
        }
        const bool below_c = draw_point<KIND>(probe, delta, seed, instance, u_sys) < c;
        const uint64_t mask = __ballot(below_c);
        // probes are increasing and x is non-decreasing: the true ones are a prefix
        const int ntrue = __popcll(mask);
        const int64_t p_last = __shfl(probe, ntrue > 0 ? ntrue - 1 : 0, kWave);
        const int64_t p_next = __shfl(probe, ntrue < kWave ? ntrue : kWave - 1, kWave);
        if (ntrue > 0) a = p_last + 1;
        if (ntrue < kWave) b = p_next;
    }
    *bad = 1;
    return a;
}

// In-tile cumulative weights C'_j (see the file comment) for tile t; every
// thread computes its four consecutive entries and stores them in Cs.
__device__ void tile_cumulative(const float *__restrict__ lw, int64_t P, int64_t t, float m,
                                double Blo, double Bhi, double *Cs, double *red,
                                double *sh_total, double Cout[4])
{
    float v[4];
    load_tile4(lw, P, t, v);
    double w[4], L[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) w[k] = exp((double)v[k] - (double)m);
    L[0] = w[0];
    L[1] = L[0] + w[1];
    L[2] = L[1] + w[2];
    L[3] = L[2] + w[3];
    double total;
    const double prefix = block_exclusive_sum(L[3], red, &total);
    // zero-weight-aware running maximum: a zero weight repeats its predecessor
    double V[4];
    double run = 0.0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if (w[k] > 0.0) run = prefix + L[k];
        V[k] = run;
    }
    const double carry = block_exclusive_max(run, red);
#pragma unroll
    for (int k = 0; k < 4; ++k) V[k] = fmax(V[k], carry);
    if (threadIdx.x == kTileThreads - 1) *sh_total = V[3];
    __syncthreads();
    const double Ltot = *sh_total;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const double C = (V[k] == Ltot) ? Bhi : fmin(Blo + V[k], Bhi);
        Cout[k] = C;
        Cs[4 * threadIdx.x + k] = C;
    }
    __syncthreads();
}

// First index j of the 1024-entry Cs with Cs[j] > x (Cs is non-decreasing).
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

// ------------------------------------------------------ launch 2: fill
template <int KIND>
__global__ __launch_bounds__(kTileThreads) void fill_kernel(const float *__restrict__ lw,
                                                            int32_t *__restrict__ anc, int64_t P,
                                                            uint64_t seed, uint32_t instance,
                                                            double *cumw, char *ws_raw,
                                                            int32_t *status)
{
    __shared__ double Cs[kTile];
    __shared__ double red[kWaves];
    __shared__ double sh_total;
    __shared__ int64_t sh_n[2];
    __shared__ int sh_bad;
    const WsView ws = ws_view(ws_raw, P, false);
    const int64_t n = num_tiles(P);
    const int64_t g = blockIdx.x;
    const int flags = ws.h->flags;
    if (flags) {  // flagged input: identity ancestors
        if (g < n) {
            for (int64_t j = g * kTile + threadIdx.x; j < min(P, (g + 1) * kTile); j += kTileThreads) {
                anc[j] = (int32_t)j;
                if (cumw) cumw[j] = (double)NAN;
            }
        }
        return;
    }
    int64_t t, c;
    if (g < n) {
        t = g;
        c = 0;
    } else {
        const int64_t q = g - n;
        if (q >= ws.h->n_overflow) return;
        int64_t lo = 0, hi = n - 1;  // last t with overflow[t] <= q
        while (lo < hi) {
            const int64_t mid = (lo + hi + 1) >> 1;
            if (ws.overflow[mid] <= q) lo = mid;
            else hi = mid - 1;
        }
        t = lo;
        c = q - ws.overflow[t] + 1;
    }
    const double W = ws.h->W, delta = ws.h->delta;
    const float m = ws.h->m;
    const double Blo = t > 0 ? ws.bound[t - 1] : 0.0;
    const double Bhi = ws.bound[t];
    double u_sys = 0.0;
    if (KIND == kSystematic) u_sys = unit32(philox(seed, 0u, instance, 0u, kTagSystematic).r0);

    if (threadIdx.x == 0) sh_bad = 0;
    __syncthreads();
    if (wave_id() < 2) {
        int bad = 0;
        const double cb = wave_id() == 0 ? Blo : Bhi;
        const int64_t N = count_below<KIND>(cb, P, W, delta, seed, instance, u_sys, &bad);
        if (lane_id() == 0) {
            sh_n[wave_id()] = N;
            if (bad) sh_bad = 1;
        }
    }
    double C[4];
    tile_cumulative(lw, P, t, m, Blo, Bhi, Cs, red, &sh_total, C);  // ends with a barrier
    if (cumw && c == 0) store_cumw(cumw, P, t, C);
    const int64_t lo = sh_n[0], hi = sh_n[1];
    const int64_t a0 = (lo & ~(int64_t)3) + c * kChunk;
    const int64_t ob = max(lo, a0), oe = min(hi, a0 + kChunk);
    if (threadIdx.x == 0) {
        // invariants: every output of the tile is covered by one of its chunks,
        // and the launch has a block for every chunk
        const int64_t last_c = ws.overflow[t + 1] - ws.overflow[t];
        if (sh_bad || (c == last_c && a0 + kChunk < hi) || lo > hi ||
            (c == 0 && ws.h->n_overflow > max_overflow_chunks(P)))
            raise_flags(status, kFlagInternal);
    }
    if (ob >= oe) return;

    const int64_t o0 = a0 + 8 * (int64_t)threadIdx.x;
    if (o0 + 8 <= ob || o0 >= oe) return;
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
    int32_t a[8];
    const int32_t tile_base = (int32_t)(t * kTile);
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const double x = ((double)(o0 + k) + U[k]) * delta;
        a[k] = tile_base + search_tile(Cs, fmin(x, cap));
    }
    const bool full = (o0 >= ob) && (o0 + 8 <= oe) && ((((uintptr_t)anc) & 15) == 0);
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

// ------------------------------------------------------ multinomial
// Launch 2m: one block per tile writes C' for the tile.
__global__ __launch_bounds__(kTileThreads) void cumulative_kernel(const float *__restrict__ lw,
                                                                  int64_t P, double *C,
                                                                  char *ws_raw)
{
    __shared__ double Cs[kTile];
    __shared__ double red[kWaves];
    __shared__ double sh_total;
    const WsView ws = ws_view(ws_raw, P, false);
    const int64_t t = blockIdx.x;
    if (ws.h->flags) {
        const int64_t base = t * kTile + 4 * (int64_t)threadIdx.x;
        for (int k = 0; k < 4; ++k)
            if (base + k < P) C[base + k] = (double)NAN;
        return;
    }
    const double Blo = t > 0 ? ws.bound[t - 1] : 0.0;
    double Cv[4];
    tile_cumulative(lw, P, t, ws.h->m, Blo, ws.bound[t], Cs, red, &sh_total, Cv);
    store_cumw(C, P, t, Cv);
}

// Launch 3m: each thread draws two points (one Philox block) and locates
// each by bisection over the tile boundaries (staged in LDS when they fit),
// then over the tile's cumulative weights.
__global__ __launch_bounds__(256) void multinomial_search_kernel(const double *__restrict__ C,
                                                                 int32_t *__restrict__ anc,
                                                                 int64_t P, uint64_t seed,
                                                                 uint32_t instance, char *ws_raw,
                                                                 int lds_bounds)
{
    extern __shared__ double sh_bound[];
    const WsView ws = ws_view(ws_raw, P, false);
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
    switch (kind) {
    case kStratified:
        hipLaunchKernelGGL(tile_reduce_kernel<kStratified>, dim3(n), tb, 0, stream, lw, P, w,
                           status, (double *)nullptr);
        hipLaunchKernelGGL(fill_kernel<kStratified>, dim3(n + max_overflow_chunks(P)), tb, 0,
                           stream, lw, anc, P, seed, instance, cumw, w, status);
        break;
    case kSystematic:
        hipLaunchKernelGGL(tile_reduce_kernel<kSystematic>, dim3(n), tb, 0, stream, lw, P, w,
                           status, (double *)nullptr);
        hipLaunchKernelGGL(fill_kernel<kSystematic>, dim3(n + max_overflow_chunks(P)), tb, 0,
                           stream, lw, anc, P, seed, instance, cumw, w, status);
        break;
    case kMultinomial: {
        double *C = cumw ? cumw : reinterpret_cast<double *>(w + ws_layout(P, true).cumw);
        hipLaunchKernelGGL(tile_reduce_kernel<kMultinomial>, dim3(n), tb, 0, stream, lw, P, w,
                           status, (double *)nullptr);
        hipLaunchKernelGGL(cumulative_kernel, dim3(n), tb, 0, stream, lw, P, C, w);
        const int lds_bounds = n <= 4096 ? 1 : 0;
        const size_t smem = lds_bounds ? (size_t)n * sizeof(double) : 0;
        const int64_t pairs = (P + 1) >> 1;
        int64_t grid = (pairs + 255) / 256;
        if (grid > 8192) grid = 8192;
        hipLaunchKernelGGL(multinomial_search_kernel, dim3(grid), dim3(256), smem, stream, C, anc,
                           P, seed, instance, w, lds_bounds);
        break;
    }
    default:
        return -1;
    }
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

int launch_log_sum_exp(const float *lw, int64_t P, double *out, void *ws, int32_t *status,
                       hipStream_t stream)
{
    hipLaunchKernelGGL(tile_reduce_kernel<kLogSumExp>, dim3(num_tiles(P)), dim3(kTileThreads), 0,
                       stream, lw, P, static_cast<char *>(ws), status, out);
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

}  // namespace rs
