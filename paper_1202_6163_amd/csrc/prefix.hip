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
//  2. table_kernel (one 1024-thread block) rescales the tile sums to the
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

namespace rs {
namespace {

// ---------------------------------------------------------------- block ops
// Called by every thread of a block of NW waves; `red` holds NW entries.
template <int NW>
__device__ double block_sum(double v, double *red)
{
    v = wave_sum(v);
    if (lane_id() == 0) red[wave_id()] = v;
    __syncthreads();
    double s = red[0];
    for (int w = 1; w < NW; ++w) s += red[w];
    __syncthreads();
    return s;
}

template <int NW>
__device__ float block_max(float v, float *red)
{
    v = wave_max(v);
    if (lane_id() == 0) red[wave_id()] = v;
    __syncthreads();
    float s = red[0];
    for (int w = 1; w < NW; ++w) s = fmaxf(s, red[w]);
    __syncthreads();
    return s;
}

template <int NW>
__device__ int block_or(int v, int *red)
{
    v = wave_or(v);
    if (lane_id() == 0) red[wave_id()] = v;
    __syncthreads();
    int s = 0;
    for (int w = 0; w < NW; ++w) s |= red[w];
    __syncthreads();
    return s;
}

// Exclusive prefix sum over threads.
template <int NW>
__device__ double block_exclusive_sum(double v, double *red)
{
    const int lane = lane_id(), wave = wave_id();
    const double incl = wave_inclusive_sum(v);
    double excl = __shfl_up(incl, 1, kWave);
    if (lane == 0) excl = 0.0;
    if (lane == kWave - 1) red[wave] = incl;
    __syncthreads();
    double wp = 0.0;
    for (int w = 0; w < wave; ++w) wp += red[w];
    __syncthreads();
    return wp + excl;
}

// Exclusive prefix maximum over threads of non-negative values (0 first).
template <int NW>
__device__ double block_exclusive_max(double v, double *red)
{
    const int lane = lane_id(), wave = wave_id();
    double incl = v;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        const double y = __shfl_up(incl, off, kWave);
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

template <int NW>
__device__ int64_t block_exclusive_isum(int64_t v, int64_t *red, int64_t *total)
{
    const int lane = lane_id(), wave = wave_id();
    int64_t incl = v;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        const int64_t y = __shfl_up(incl, off, kWave);
        if (lane >= off) incl += y;
    }
    int64_t excl = __shfl_up(incl, 1, kWave);
    if (lane == 0) excl = 0;
    if (lane == kWave - 1) red[wave] = incl;
    __syncthreads();
    int64_t wp = 0, tot = 0;
    for (int w = 0; w < NW; ++w) {
        if (w < wave) wp += red[w];
        tot += red[w];
    }
    __syncthreads();
    *total = tot;
    return wp + excl;
}

constexpr int kTileWaves = kTileThreads / kWave;
constexpr int kTableWaves = kTableThreads / kWave;

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
    int32_t *overflow;
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
    v.overflow = reinterpret_cast<int32_t *>(ws + L.overflow);
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

// Draw points x_i for i = w0 .. w0 + 11, w0 a multiple of 4 (three Philox
// blocks for stratified draws, computed side by side).
template <int KIND>
__device__ __forceinline__ void draw_window(int64_t w0, double delta, uint64_t seed,
                                            uint32_t instance, double u_sys, double x[12])
{
    if (KIND == kStratified) {
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const Block4 b = philox(seed, (uint32_t)(w0 >> 2) + (uint32_t)q, instance, 0u,
                                    kTagStratified);
            const double u[4] = {unit32(b.r0), unit32(b.r1), unit32(b.r2), unit32(b.r3)};
#pragma unroll
            for (int k = 0; k < 4; ++k) x[4 * q + k] = ((double)(w0 + 4 * q + k) + u[k]) * delta;
        }
    } else {
#pragma unroll
        for (int k = 0; k < 12; ++k) x[k] = ((double)(w0 + k) + u_sys) * delta;
    }
}

// N(c) = #{i : x_i < c} for the non-decreasing stratified/systematic draw
// points, or P when c >= W (draws at or past W belong to the last positive
// tile). The answer lies within a couple of strata of c / (W/P); a window of
// twelve draws there settles it, and a bisection over all P covers the rest.
template <int KIND>
__device__ int64_t count_below(double c, int64_t P, double W, double delta, uint64_t seed,
                               uint32_t instance, double u_sys)
{
    if (c >= W) return P;
    if (!(c > 0.0)) return 0;
    const double est = floor(c / delta);
    const int64_t s = est < 3.0 ? 0 : (est > (double)P ? P : (int64_t)est - 3);
    const int64_t w0 = s & ~(int64_t)3;
    double x[12];
    draw_window<KIND>(w0, delta, seed, instance, u_sys, x);
    if (w0 == 0 || x[0] < c) {
        // every draw before the window is below c: the answer is the first
        // window draw >= c, if the window holds one
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            if (w0 + k >= P) return P;
            if (x[k] >= c) return w0 + k;
        }
    }
    // fallback (not expected): bisection, one draw per step
    int64_t lo = 0, hi = P;
    while (lo < hi) {
        const int64_t mid = lo + ((hi - lo) >> 1);
        if (draw_point<KIND>(mid, delta, seed, instance, u_sys) < c) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// ------------------------------------------------------ launch 1: tiles
__global__ __launch_bounds__(kTileThreads) void tile_reduce_kernel(const float *__restrict__ lw,
                                                                   int64_t P, char *ws_raw)
{
    __shared__ double redd[kTileWaves];
    __shared__ float redf[kTileWaves];
    __shared__ int redi[kTileWaves];
    const WsView ws = ws_view(ws_raw, P);
    const int64_t t = blockIdx.x;
    float v[4];
    load_tile4(lw, P, t, v);
    int fl = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if (isnan(v[k])) fl |= kFlagNan;
        else if (isinf(v[k]) && v[k] > 0.0f) fl |= kFlagPosInf;
    }
    const float mx = block_max<kTileWaves>(fmaxf(fmaxf(v[0], v[1]), fmaxf(v[2], v[3])), redf);
    fl = block_or<kTileWaves>(fl, redi);
    double s = 0.0;
    if (mx > -INFINITY) {
#pragma unroll
        for (int k = 0; k < 4; ++k) s += exp((double)v[k] - (double)mx);
    }
    s = block_sum<kTileWaves>(s, redd);
    if (threadIdx.x == 0) {
        ws.tile_max[t] = mx;
        ws.tile_sum[t] = s;
        ws.tile_flags[t] = fl;
    }
}

// ------------------------------------------------------ launch 2: table
// The per-tile arrays live in LDS when they fit (kTableLdsTiles tiles),
// otherwise in the workspace; either way every value is computed by the same
// operations in the same order.
constexpr int64_t kTableLdsTiles = 4096;

template <int KIND, bool LDS>
__global__ __launch_bounds__(kTableThreads) void table_kernel(int64_t P, uint64_t seed,
                                                              uint32_t instance, char *ws_raw,
                                                              int32_t *status, double *lse_out)
{
    __shared__ double redd[kTableWaves];
    __shared__ float redf[kTableWaves];
    __shared__ int redi[kTableWaves];
    __shared__ int64_t redl[kTableWaves];
    __shared__ double sh_W;
    extern __shared__ double sh_tab[];  // [n] boundaries, then [n] counts
    const WsView ws = ws_view(ws_raw, P);
    WsHeader *h = ws.h;
    const int64_t n = num_tiles(P);
    const int tid = threadIdx.x;
    double *bound = LDS ? sh_tab : ws.bound;
    int32_t *count = LDS ? reinterpret_cast<int32_t *>(sh_tab + n) : ws.count;
    // each thread owns a contiguous run of tiles
    const int64_t per = (n + kTableThreads - 1) / kTableThreads;
    const int64_t t0 = min(n, (int64_t)tid * per), t1 = min(n, t0 + per);

    int fl = 0;
    float m = -INFINITY;
    for (int64_t t = t0; t < t1; ++t) {
        fl |= ws.tile_flags[t];
        const float mt = ws.tile_max[t];
        m = fmaxf(m, mt);
        bound[t] = ws.tile_sum[t];  // staged next to the max
    }
    fl = block_or<kTableWaves>(fl, redi);
    m = block_max<kTableWaves>(m, redf);
    if (!(m > -INFINITY)) fl |= kFlagAllNegInf;
    if (fl) {
        if (tid == 0) {
            h->flags = fl;
            h->n_overflow = 0;
            if (lse_out)
                *lse_out = (fl & (kFlagNan | kFlagPosInf)) ? (double)NAN : -(double)INFINITY;
            raise_flags(status, fl);
        }
        return;
    }

    // tile sums rescaled to the global max, scanned, then made non-decreasing
    double local = 0.0;
    for (int64_t t = t0; t < t1; ++t) {
        const float mt = ws.tile_max[t];
        const double S = (mt > -INFINITY) ? bound[t] * exp((double)mt - (double)m) : 0.0;
        bound[t] = S;
        local += S;
    }
    double run = block_exclusive_sum<kTableWaves>(local, redd);
    double tmax = 0.0;
    for (int64_t t = t0; t < t1; ++t) {
        run += bound[t];
        bound[t] = run;
        tmax = run;  // running sums grow within a thread
    }
    const double carry = block_exclusive_max<kTableWaves>(tmax, redd);
    for (int64_t t = t0; t < t1; ++t) {
        const double b = fmax(bound[t], carry);
        bound[t] = b;
        if (LDS) ws.bound[t] = b;
        if (t == n - 1) sh_W = b;
    }
    __syncthreads();
    const double W = sh_W;
    const double delta = W / (double)P;

    if (KIND == kStratified || KIND == kSystematic) {
        const double u_sys =
            KIND == kSystematic ? unit32(philox(seed, 0u, instance, 0u, kTagSystematic).r0) : 0.0;
        for (int64_t t = t0; t < t1; ++t) {
            const int32_t cnt =
                (int32_t)count_below<KIND>(bound[t], P, W, delta, seed, instance, u_sys);
            count[t] = cnt;
            if (LDS) ws.count[t] = cnt;
        }
        __syncthreads();  // counts of the previous thread's last tile are visible
        // fill blocks per tile: ceil((hi - (lo & ~3)) / kChunk), at least one
        int64_t nov = 0;
        for (int64_t t = t0; t < t1; ++t) {
            const int64_t lo = t > 0 ? count[t - 1] : 0, hi = count[t];
            const int64_t span = hi - (lo & ~(int64_t)3);
            nov += span > kChunk ? (span + kChunk - 1) / kChunk - 1 : 0;
        }
        int64_t tot_ov;
        int64_t acc = block_exclusive_isum<kTableWaves>(nov, redl, &tot_ov);
        for (int64_t t = t0; t < t1; ++t) {
            ws.overflow[t] = (int32_t)acc;
            const int64_t lo = t > 0 ? count[t - 1] : 0, hi = count[t];
            const int64_t span = hi - (lo & ~(int64_t)3);
            acc += span > kChunk ? (span + kChunk - 1) / kChunk - 1 : 0;
        }
        if (tid == 0) {
            ws.overflow[n] = (int32_t)tot_ov;
            h->n_overflow = (int32_t)tot_ov;
            if (tot_ov > max_overflow_chunks(P)) raise_flags(status, kFlagInternal);
        }
    }
    if (tid == 0) {
        h->m = m;
        h->W = W;
        h->delta = delta;
        h->lse = (double)m + log(W);
        h->flags = 0;
        if (lse_out) *lse_out = h->lse;
    }
}

template <int KIND>
void launch_table(int64_t P, uint64_t seed, uint32_t instance, char *w, int32_t *status,
                  double *lse_out, hipStream_t stream)
{
    const int64_t n = num_tiles(P);
    if (n <= kTableLdsTiles) {
        const size_t smem = (size_t)n * (sizeof(double) + sizeof(int32_t));
        hipLaunchKernelGGL((table_kernel<KIND, true>), dim3(1), dim3(kTableThreads), smem, stream,
                           P, seed, instance, w, status, lse_out);
    } else {
        hipLaunchKernelGGL((table_kernel<KIND, false>), dim3(1), dim3(kTableThreads), 0, stream, P,
                           seed, instance, w, status, lse_out);
    }
}

// In-tile cumulative weights C'_j (see the file comment) from the thread's
// four log-weights v; every thread stores its four entries in Cs.
__device__ void tile_cumulative(const float v[4], float m, double Blo, double Bhi, double *Cs,
                                double *red, double *sh_total, double Cout[4])
{
    double w[4], L[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) w[k] = exp((double)v[k] - (double)m);
    L[0] = w[0];
    L[1] = L[0] + w[1];
    L[2] = L[1] + w[2];
    L[3] = L[2] + w[3];
    const double prefix = block_exclusive_sum<kTileWaves>(L[3], red);
    // zero-weight-aware running maximum: a zero weight repeats its predecessor
    double V[4];
    double run = 0.0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if (w[k] > 0.0) run = prefix + L[k];
        V[k] = run;
    }
    const double carry = block_exclusive_max<kTileWaves>(run, red);
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

// ------------------------------------------------------ launch 3: fill
template <int KIND>
__global__ __launch_bounds__(kTileThreads) void fill_kernel(const float *__restrict__ lw,
                                                            int32_t *__restrict__ anc, int64_t P,
                                                            uint64_t seed, uint32_t instance,
                                                            double *cumw, char *ws_raw)
{
    __shared__ double Cs[kTile];
    __shared__ double red[kTileWaves];
    __shared__ double sh_total;
    const WsView ws = ws_view(ws_raw, P);
    const int64_t n = num_tiles(P);
    const int64_t g = blockIdx.x;
    int64_t t = g, c = 0;
    float v[4];
    // every read this block needs is issued up front (one memory round trip)
    const int64_t tq = g < n ? g : n - 1;
    load_tile4(lw, P, tq, v);
    const int flags = ws.h->flags;
    const int n_ov = ws.h->n_overflow;
    const double delta = ws.h->delta;
    const float m = ws.h->m;
    int64_t lo = tq > 0 ? ws.count[tq - 1] : 0, hi = ws.count[tq];
    double Blo = tq > 0 ? ws.bound[tq - 1] : 0.0, Bhi = ws.bound[tq];
    if (flags) {  // flagged input: identity ancestors
        if (g < n) {
            for (int64_t j = g * kTile + threadIdx.x; j < min(P, (g + 1) * kTile); j += kTileThreads) {
                anc[j] = (int32_t)j;
                if (cumw) cumw[j] = (double)NAN;
            }
        }
        return;
    }
    if (g >= n) {
        const int64_t q = g - n;
        if (q >= n_ov) return;
        int64_t a = 0, z = n - 1;  // last t with overflow[t] <= q
        while (a < z) {
            const int64_t mid = (a + z + 1) >> 1;
            if (ws.overflow[mid] <= q) a = mid;
            else z = mid - 1;
        }
        t = a;
        c = q - ws.overflow[t] + 1;
        load_tile4(lw, P, t, v);
        lo = t > 0 ? ws.count[t - 1] : 0;
        hi = ws.count[t];
        Blo = t > 0 ? ws.bound[t - 1] : 0.0;
        Bhi = ws.bound[t];
    }
    const int64_t a0 = (lo & ~(int64_t)3) + c * kChunk;
    const int64_t ob = max(lo, a0), oe = min(hi, a0 + kChunk);
    if (ob >= oe && !(cumw && c == 0)) return;  // nothing to write

    double C[4];
    tile_cumulative(v, m, Blo, Bhi, Cs, red, &sh_total, C);  // ends with a barrier
    if (cumw && c == 0) store_cumw(cumw, P, t, C);

    const int64_t o0 = a0 + 8 * (int64_t)threadIdx.x;
    if (o0 + 8 <= ob || o0 >= oe) return;
    double U[8];
    if (KIND == kStratified) {
        const Block4 b0 = philox(seed, (uint32_t)(o0 >> 2), instance, 0u, kTagStratified);
        const Block4 b1 = philox(seed, (uint32_t)(o0 >> 2) + 1u, instance, 0u, kTagStratified);
        U[0] = unit32(b0.r0); U[1] = unit32(b0.r1); U[2] = unit32(b0.r2); U[3] = unit32(b0.r3);
        U[4] = unit32(b1.r0); U[5] = unit32(b1.r1); U[6] = unit32(b1.r2); U[7] = unit32(b1.r3);
    } else {
        const double u_sys = unit32(philox(seed, 0u, instance, 0u, kTagSystematic).r0);
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
// Launch 3m: one block per tile writes C' for the tile.
__global__ __launch_bounds__(kTileThreads) void cumulative_kernel(const float *__restrict__ lw,
                                                                  int64_t P, double *C,
                                                                  char *ws_raw)
{
    __shared__ double Cs[kTile];
    __shared__ double red[kTileWaves];
    __shared__ double sh_total;
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
    tile_cumulative(v, ws.h->m, Blo, ws.bound[t], Cs, red, &sh_total, Cv);
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
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

int launch_log_sum_exp(const float *lw, int64_t P, double *out, void *ws, int32_t *status,
                       hipStream_t stream)
{
    char *w = static_cast<char *>(ws);
    hipLaunchKernelGGL(tile_reduce_kernel, dim3((uint32_t)num_tiles(P)), dim3(kTileThreads), 0,
                       stream, lw, P, w);
    launch_table<kLogSumExp>(P, 0, 0u, w, status, out, stream);
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

}  // namespace rs
