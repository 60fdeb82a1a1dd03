// Sorted-weight variants of the prefix-sum resamplers (Sec. 3 of the paper:
// the weights are sorted before the prefix sum, which shortens the
// multinomial bisection; the paper finds the sort costs more than it saves).
//
// Steps: the log-weights are sorted in decreasing order, equal weights in
// index order (-0 as +0), by a stable least-significant-digit radix sort
// written here, which carries the particle indices along; the chosen
// resampler runs on the sorted weights; ancestors are mapped back through the
// permutation. Flagged inputs give identity ancestors, as the plain
// resamplers do.
//
// Radix sort: four passes of eight bits over a 32-bit key whose ascending
// order is the weights' descending order. Up to 4096 particles one block
// sorts everything in LDS. Beyond, each pass counts the digits of every
// 4096-element block of its input into a 256-bin LDS histogram, turns the
// histograms into each block's starting position per digit in digit-major
// order (digit d of block b starts after every smaller digit and after digit
// d of every earlier block: up to 64 blocks each scatter block sums the
// counts it needs itself, beyond that one scan launch does it), and
// scatters: each block walks its elements in index order, 256 at a time,
// and ranks every element among the equal digits before it (peers within a
// wave from eight ballots, waves before it from per-wave counts in LDS).
// Equal keys therefore keep their order in every pass, and the sort is
// stable. The first pass reads the log-weights themselves and numbers the
// particles.
#include <hip/hip_runtime.h>

#include "common.h"
#include "launch.h"
#include "prefix.h"

namespace rs {
namespace {

constexpr int kThreads = 256;                           // the map-back kernel
constexpr int kSortThreads = 1024;                      // the sort kernels
constexpr int kSortItems = 4;                           // elements per thread and block
constexpr int kSortBlock = kSortThreads * kSortItems;   // 4096 elements per block
constexpr int kRadix = 256;                             // eight bits per pass
constexpr int kPasses = 4;                              // 32-bit keys
constexpr int64_t kOwnScanBlocks = 64;                  // up to this many blocks, no scan launch
constexpr int kSortWaves = kSortThreads / kWave;
constexpr int kDigitWaves = kRadix / kWave;             // the waves that own a digit each lane
static_assert(kRadix <= kSortThreads && kRadix % kWave == 0, "threads 0..255 own the digits");

// A key whose ascending order is the descending order of the log-weight,
// -0 equal to +0 (the IEEE order made unsigned, then reversed).
__device__ __forceinline__ uint32_t sort_key(float v)
{
    const uint32_t b = __float_as_uint(v == 0.0f ? 0.0f : v);
    const uint32_t f = (b & 0x80000000u) ? ~b : (b | 0x80000000u);
    return ~f;
}

// One pass's histograms: hist[digit][block].
__global__ __launch_bounds__(kSortThreads) void radix_hist_kernel(const float *__restrict__ keys,
                                                                  int64_t P, int shift,
                                                                  uint32_t *__restrict__ hist,
                                                                  int64_t nblk)
{
    __shared__ uint32_t h[kRadix];
    const int tid = threadIdx.x;
    if (tid < kRadix) h[tid] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kSortBlock;
#pragma unroll
    for (int k = 0; k < kSortItems; ++k) {
        const int64_t i = base + k * kSortThreads + tid;
        if (i < P) atomicAdd(&h[(sort_key(keys[i]) >> shift) & (kRadix - 1)], 1u);
    }
    __syncthreads();
    if (tid < kRadix) hist[(int64_t)tid * nblk + blockIdx.x] = h[tid];
}

// Exclusive scan in place of n counts (one block; totals stay below 2^31).
__global__ __launch_bounds__(1024) void radix_scan_kernel(uint32_t *__restrict__ c, int64_t n)
{
    __shared__ uint32_t red[1024 / kWave];
    const int tid = threadIdx.x, lane = lane_id(), wave = wave_id();
    const int64_t per = (n + 1023) / 1024;
    const int64_t t0 = min(n, tid * per), t1 = min(n, t0 + per);
    uint32_t sum = 0;
    for (int64_t q = t0; q < t1; ++q) sum += c[q];
    const uint32_t incl = wave_scan(sum, 0u, AddOp{});
    if (lane == kWave - 1) red[wave] = incl;
    __syncthreads();
    uint32_t run = incl - sum;
    for (int w = 0; w < wave; ++w) run += red[w];
    for (int64_t q = t0; q < t1; ++q) {
        const uint32_t v = c[q];
        c[q] = run;
        run += v;
    }
}

// FIRST: kin is the log-weights (-0 stored as +0) and the values are the
// particle indices. OWN_SCAN: offs holds the raw histograms and the block
// forms its starting positions itself (few blocks); else offs holds them
// already scanned.
template <bool FIRST, bool OWN_SCAN>
__global__ __launch_bounds__(kSortThreads) void radix_scatter_kernel(
    const float *__restrict__ kin, const int32_t *__restrict__ vin, float *__restrict__ kout,
    int32_t *__restrict__ vout, int64_t P, int shift, const uint32_t *__restrict__ offs,
    int64_t nblk)
{
    __shared__ uint32_t next[kRadix];              // next output position per digit
    __shared__ uint32_t wcnt[kSortWaves][kRadix];  // this round's count per wave and digit
    __shared__ uint32_t wtot[kDigitWaves];
    const int tid = threadIdx.x, lane = lane_id(), wave = wave_id();
    if (OWN_SCAN) {
        // digit tid: its count in the earlier blocks and in all blocks
        uint32_t before = 0, total = 0;
        if (tid < kRadix) {
            const uint32_t *row = offs + (int64_t)tid * nblk;
            for (int64_t b = 0; b < nblk; ++b) {
                const uint32_t c = row[b];
                before += b < (int64_t)blockIdx.x ? c : 0u;
                total += c;
            }
        }
        // the smaller digits' totals: an exclusive scan over digits (waves
        // beyond the digits scan zeros)
        const uint32_t incl = wave_scan(total, 0u, AddOp{});
        if (lane == kWave - 1 && wave < kDigitWaves) wtot[wave] = incl;
        __syncthreads();
        if (tid < kRadix) {
            uint32_t smaller = incl - total;
            for (int w = 0; w < wave; ++w) smaller += wtot[w];
            next[tid] = smaller + before;
        }
    } else if (tid < kRadix) {
        next[tid] = offs[(int64_t)tid * nblk + blockIdx.x];
    }
    for (int e = tid; e < kSortWaves * kRadix; e += kSortThreads) (&wcnt[0][0])[e] = 0;
    __syncthreads();
    const uint64_t below = (1ull << lane) - 1ull;
    const int64_t base = (int64_t)blockIdx.x * kSortBlock;
    for (int r = 0; r < kSortItems; ++r) {
        const int64_t i = base + r * kSortThreads + tid;  // index order: round, then thread
        const bool valid = i < P;
        float key = valid ? kin[i] : 0.0f;
        if (FIRST && key == 0.0f) key = 0.0f;  // -0 as +0
        const int32_t val = FIRST ? (int32_t)i : (valid ? vin[i] : 0);
        const uint32_t d = (sort_key(key) >> shift) & (kRadix - 1);
        // the lanes of this wave with the same digit (valid ones only)
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int bit = 0; bit < 8; ++bit) {
            const bool on = (d >> bit) & 1u;
            const uint64_t m = __ballot(on);
            peers &= on ? m : ~m;
        }
        if (valid && (peers & below) == 0) wcnt[wave][d] = (uint32_t)__popcll(peers);
        __syncthreads();
        if (valid) {
            uint32_t pos = next[d] + (uint32_t)__popcll(peers & below);
            for (int w = 0; w < wave; ++w) pos += wcnt[w][d];
            kout[pos] = key;
            vout[pos] = val;
        }
        __syncthreads();
        if (tid < kRadix) {
            uint32_t add = 0;
#pragma unroll
            for (int w = 0; w < kSortWaves; ++w) {
                add += wcnt[w][tid];
                wcnt[w][tid] = 0;
            }
            next[tid] += add;
        }
        __syncthreads();
    }
}

// Up to kSortBlock particles: the whole sort in one block, keys and indices
// in LDS (two buffers of kSortBlock each, dynamic), the same four stable
// passes; writes the sorted keys and indices to kout, vout.
__global__ __launch_bounds__(kSortThreads) void radix_block_kernel(const float *__restrict__ lw,
                                                                   int64_t P,
                                                                   float *__restrict__ kout,
                                                                   int32_t *__restrict__ vout)
{
    extern __shared__ uint32_t lds[];  // two buffers of transformed keys, then two of indices
    __shared__ uint32_t next[kRadix];
    __shared__ uint32_t wcnt[kSortWaves][kRadix];
    __shared__ uint32_t wtot[kDigitWaves];
    const int tid = threadIdx.x, lane = lane_id(), wave = wave_id();
    const int n = (int)P;
    for (int i = tid; i < n; i += kSortThreads) {
        lds[i] = sort_key(lw[i]);
        lds[2 * kSortBlock + i] = (uint32_t)i;
    }
    for (int e = tid; e < kSortWaves * kRadix; e += kSortThreads) (&wcnt[0][0])[e] = 0;
    const uint64_t below = (1ull << lane) - 1ull;
    int cur = 0;
    for (int shift = 0; shift < 32; shift += 8, cur ^= 1) {
        const uint32_t *ki = lds + cur * kSortBlock, *vi = lds + (2 + cur) * kSortBlock;
        uint32_t *ko = lds + (cur ^ 1) * kSortBlock, *vo = lds + (2 + (cur ^ 1)) * kSortBlock;
        if (tid < kRadix) next[tid] = 0;
        __syncthreads();
        for (int i = tid; i < n; i += kSortThreads) atomicAdd(&next[(ki[i] >> shift) & 255u], 1u);
        __syncthreads();
        {
            const uint32_t c = tid < kRadix ? next[tid] : 0u;
            const uint32_t incl = wave_scan(c, 0u, AddOp{});
            if (lane == kWave - 1 && wave < kDigitWaves) wtot[wave] = incl;
            __syncthreads();
            if (tid < kRadix) {
                uint32_t ex = incl - c;
                for (int w = 0; w < wave; ++w) ex += wtot[w];
                next[tid] = ex;
            }
            __syncthreads();
        }
        for (int r = 0; r * kSortThreads < n; ++r) {
            const int i = r * kSortThreads + tid;
            const bool valid = i < n;
            const uint32_t k = valid ? ki[i] : 0u;
            const uint32_t v = valid ? vi[i] : 0u;
            const uint32_t d = (k >> shift) & 255u;
            uint64_t peers = __ballot(valid);
#pragma unroll
            for (int bit = 0; bit < 8; ++bit) {
                const bool on = (d >> bit) & 1u;
                const uint64_t m = __ballot(on);
                peers &= on ? m : ~m;
            }
            if (valid && (peers & below) == 0) wcnt[wave][d] = (uint32_t)__popcll(peers);
            __syncthreads();
            if (valid) {
                uint32_t pos = next[d] + (uint32_t)__popcll(peers & below);
                for (int w = 0; w < wave; ++w) pos += wcnt[w][d];
                ko[pos] = k;
                vo[pos] = v;
            }
            __syncthreads();
            if (tid < kRadix) {
                uint32_t add = 0;
#pragma unroll
                for (int w = 0; w < kSortWaves; ++w) {
                    add += wcnt[w][tid];
                    wcnt[w][tid] = 0;
                }
                next[tid] += add;
            }
            __syncthreads();
        }
    }
    // four passes: back in buffer 0; the keys go out as the log-weights
    // (-0 as +0), recovered from the transform
    for (int i = tid; i < n; i += kSortThreads) {
        const uint32_t f = ~lds[cur * kSortBlock + i];
        const uint32_t b = (f & 0x80000000u) ? (f & 0x7FFFFFFFu) : ~f;
        kout[i] = __uint_as_float(b);
        vout[i] = (int32_t)lds[(2 + cur) * kSortBlock + i];
    }
}

__global__ __launch_bounds__(kThreads) void map_back_kernel(const int32_t *__restrict__ a_sorted,
                                                            const int32_t *__restrict__ perm,
                                                            int32_t *__restrict__ anc, int64_t P,
                                                            const WsHeader *h)
{
    const int flags = h->flags;
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < P; i += stride)
        anc[i] = flags ? (int32_t)i : perm[a_sorted[i]];
}

uint32_t grid_for(int64_t work)
{
    int64_t g = (work + kThreads - 1) / kThreads;
    return (uint32_t)(g < 1 ? 1 : (g > 16384 ? 16384 : g));
}

size_t al(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

int64_t sort_blocks(int64_t P) { return (P + kSortBlock - 1) / kSortBlock; }

SortedLayout sorted_layout(int64_t P, int kind)
{
    const size_t p = (size_t)P;
    SortedLayout L;
    L.prefix = 0;
    L.keys_in = al(ws_layout(P, kind == kMultinomial).total);
    L.keys_out = L.keys_in + al(4 * p);
    L.idx_in = L.keys_out + al(4 * p);
    L.perm = L.idx_in + al(4 * p);
    L.a_sorted = L.perm + al(4 * p);
    L.temp = L.a_sorted + al(4 * p);
    L.temp_bytes = al((size_t)kRadix * (size_t)sort_blocks(P) * sizeof(uint32_t));
    L.total = L.temp + L.temp_bytes;
    return L;
}

int launch_sorted(int kind, const float *lw, int32_t *anc, int64_t P, uint64_t seed,
                  uint32_t instance, void *ws, int32_t *status, hipStream_t stream)
{
    const SortedLayout L = sorted_layout(P, kind);
    char *w = static_cast<char *>(ws);
    float *keys[2] = {reinterpret_cast<float *>(w + L.keys_in),
                      reinterpret_cast<float *>(w + L.keys_out)};
    int32_t *idx[2] = {reinterpret_cast<int32_t *>(w + L.idx_in),
                       reinterpret_cast<int32_t *>(w + L.perm)};
    int32_t *a_sorted = reinterpret_cast<int32_t *>(w + L.a_sorted);
    uint32_t *hist = reinterpret_cast<uint32_t *>(w + L.temp);
    int cur = 0;
    if (P <= kSortBlock) {
        const size_t smem = 4 * kSortBlock * sizeof(uint32_t);
        if (allow_dynamic_lds(reinterpret_cast<const void *>(&radix_block_kernel), smem)) return -3;
        hipLaunchKernelGGL(radix_block_kernel, dim3(1), dim3(kSortThreads), smem, stream, lw, P,
                           keys[0], idx[0]);
    } else {
        const int64_t nblk = sort_blocks(P);
        const bool own = nblk <= kOwnScanBlocks;
        const float *kin = lw;
        for (int q = 0; q < kPasses; ++q) {
            const int shift = 8 * q;
            float *ko = keys[q & 1 ? 0 : 1];
            int32_t *vo = idx[q & 1 ? 0 : 1];
            const int32_t *vi = idx[q & 1 ? 1 : 0];
            hipLaunchKernelGGL(radix_hist_kernel, dim3((uint32_t)nblk), dim3(kSortThreads), 0,
                               stream, kin, P, shift, hist, nblk);
            if (!own)
                hipLaunchKernelGGL(radix_scan_kernel, dim3(1), dim3(1024), 0, stream, hist,
                                   (int64_t)kRadix * nblk);
            const dim3 g((uint32_t)nblk), tb(kSortThreads);
            if (q == 0 && own)
                hipLaunchKernelGGL((radix_scatter_kernel<true, true>), g, tb, 0, stream, kin,
                                   nullptr, ko, vo, P, shift, hist, nblk);
            else if (q == 0)
                hipLaunchKernelGGL((radix_scatter_kernel<true, false>), g, tb, 0, stream, kin,
                                   nullptr, ko, vo, P, shift, hist, nblk);
            else if (own)
                hipLaunchKernelGGL((radix_scatter_kernel<false, true>), g, tb, 0, stream, kin, vi,
                                   ko, vo, P, shift, hist, nblk);
            else
                hipLaunchKernelGGL((radix_scatter_kernel<false, false>), g, tb, 0, stream, kin,
                                   vi, ko, vo, P, shift, hist, nblk);
            kin = ko;
        }
        // passes write buffers 1, 0, 1, 0: the result is in buffer 0
    }
    // the sorted keys and their particle indices are in buffer 0 (cur)
    int rc = launch_prefix(kind, keys[cur], a_sorted, nullptr, P, seed, instance, nullptr, w,
                           status, stream);
    if (rc) return rc;
    hipLaunchKernelGGL(map_back_kernel, dim3(grid_for(P)), dim3(kThreads), 0, stream, a_sorted,
                       idx[cur], anc, P, reinterpret_cast<const WsHeader *>(w));
    return launch_status();
}

}  // namespace rs
