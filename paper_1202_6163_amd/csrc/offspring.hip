// Offspring counts from ancestors with a workspace, without device-scope
// atomics, on gfx950.
//
// Method (Sec. 2: a resampler's output as ancestors a_i or as offspring
// o_j = #{i : a_i = j}; converting between the two is a count). The plain
// conversion (offspring_kernel) adds one device-scope atomic per run of equal
// ancestors; random ancestors make that about P atomics at random addresses,
// which the eight XCDs' L2s cannot combine (they go to memory). Here the
// ancestors are first grouped by bucket of 2^12 to 2^15 particles, then each
// bucket's counts are formed in LDS and written whole:
//  1. off_hist_kernel: per block of `per` ancestors, the number falling in
//     each bucket (LDS atomics), stored bucket-major: hist[b][blk].
//  2. off_rowscan_kernel (a small block per bucket): hist[b][blk] becomes the
//     count of bucket b in the blocks before blk, tot[b] the bucket's total.
//  3. off_scatter_kernel: each block forms the buckets' starts from tot (a
//     block scan), stages each chunk of its ancestors in LDS ordered by
//     bucket and writes every bucket's run contiguously into the grouped
//     array (order inside a bucket is free, the counts do not depend on it).
//  4. off_count_kernel: block b counts bucket b's ancestors (their range
//     from the starts block 0 of the scatter wrote) in LDS (equal
//     ancestors of a wave combined first, so a particle that takes most of
//     the draws costs one LDS atomic per wave) and writes o_j for every j of
//     the bucket, zeros included: no clearing pass.
// Every value is an exact integer, so the result equals the plain
// conversion's bit for bit. Ancestors outside [0, P) raise RS_FLAG_BAD_ANCESTOR
// and are left out, as in the plain conversion.
#include <hip/hip_runtime.h>

#include "common.h"
#include "launch.h"
#include "prefix.h"

namespace rs {
namespace {

constexpr int kOffThreads = 1024;
constexpr int kOffWaves = kOffThreads / kWave;
constexpr int kRowThreads = 256;                          // the row scan: one entry per thread
constexpr int kMinBucketBits = 12, kMaxBucketBits = 15;  // 4096 .. 32768 particles per bucket
constexpr int64_t kMaxBuckets = 512;
constexpr int64_t kMaxP = kMaxBuckets << kMaxBucketBits;  // 2^24: larger P takes the atomics
constexpr int64_t kMaxHistBlocks = kRowThreads;          // blocks of the histogram and scatter
constexpr int64_t kBlockGrain = 4096;                    // ancestors per block: a multiple of this
static_assert(kMaxBuckets <= kOffThreads, "a thread per bucket in the bucket scans");

struct OffLayout {
    int bits;               // log2 of the particles per bucket
    int64_t nb, nblk, per;  // buckets, element blocks, ancestors per element block
    size_t hist, tot, bstart, grouped, total;
};

// Buckets of 2^bits particles, as few as 256 (never more than kMaxBuckets);
// at most kMaxHistBlocks blocks, each a multiple of kBlockGrain ancestors.
__host__ __device__ inline OffLayout off_layout(int64_t P)
{
    OffLayout L;
    int lg = 0;
    while ((int64_t(1) << lg) < P) ++lg;
    L.bits = lg - 8;
    L.bits = L.bits < kMinBucketBits ? kMinBucketBits : (L.bits > kMaxBucketBits ? kMaxBucketBits : L.bits);
    L.nb = (P + (int64_t(1) << L.bits) - 1) >> L.bits;
    const int64_t per = (P + kMaxHistBlocks - 1) / kMaxHistBlocks;
    L.per = (per + kBlockGrain - 1) / kBlockGrain * kBlockGrain;
    L.nblk = (P + L.per - 1) / L.per;
    L.hist = 0;
    L.tot = ws_align((size_t)(L.nb * L.nblk) * sizeof(uint32_t));
    L.bstart = L.tot + ws_align((size_t)L.nb * sizeof(uint32_t));
    L.grouped = L.bstart + ws_align((size_t)L.nb * sizeof(uint32_t));
    L.total = L.grouped + ws_align((size_t)P * sizeof(int32_t));
    return L;
}

// Exclusive prefix of v over threads 0 .. nb-1 of a kOffThreads block (the
// others pass 0); red: kOffWaves words of LDS. Ends with a barrier.
__device__ inline uint32_t bucket_excl(uint32_t v, uint32_t *red)
{
    const int lane = lane_id(), wave = wave_id();
    const uint32_t incl = wave_scan(v, 0u, AddOp{});
    if (lane == kWave - 1) red[wave] = incl;
    __syncthreads();
    uint32_t ex = incl - v;
    for (int w = 0; w < wave; ++w) ex += red[w];
    __syncthreads();
    return ex;
}

// Four consecutive ancestors from i (16-byte load when aligned and whole);
// entries at or past i1 come back as -1.
__device__ __forceinline__ void load_anc4(const int32_t *__restrict__ anc, int64_t i, int64_t i1,
                                          int32_t a[4])
{
    if (i + 3 < i1 && (((uintptr_t)(anc + i)) & 15) == 0) {
        const int4 q = *reinterpret_cast<const int4 *>(anc + i);
        a[0] = q.x, a[1] = q.y, a[2] = q.z, a[3] = q.w;
    } else {
#pragma unroll
        for (int k = 0; k < 4; ++k) a[k] = i + k < i1 ? anc[i + k] : -1;
    }
}

__global__ __launch_bounds__(kOffThreads) void off_hist_kernel(const int32_t *__restrict__ anc,
                                                               int64_t P, uint32_t *hist, int bits,
                                                               int64_t nb, int64_t nblk,
                                                               int64_t per, int32_t *status)
{
    __shared__ uint32_t h[kMaxBuckets];
    const int tid = threadIdx.x;
    for (int64_t b = tid; b < nb; b += kOffThreads) h[b] = 0;
    __syncthreads();
    const int64_t i0 = (int64_t)blockIdx.x * per, i1 = min(P, i0 + per);
    int fl = 0;
    for (int64_t i = i0 + 4 * (int64_t)tid; i < i1; i += 4 * kOffThreads) {
        int32_t a[4];
        load_anc4(anc, i, i1, a);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if (i + k >= i1) continue;
            if (a[k] < 0 || (int64_t)a[k] >= P) {
                fl |= kFlagBadAncestor;
                continue;
            }
            atomicAdd(&h[a[k] >> bits], 1u);
        }
    }
    __syncthreads();
    for (int64_t b = tid; b < nb; b += kOffThreads) hist[b * nblk + blockIdx.x] = h[b];
    raise_flags(status, fl);
}

// Block b: hist[b][0, nblk) (nblk <= kRowThreads) becomes its exclusive
// prefix, tot[b] the row's total.
__global__ __launch_bounds__(kRowThreads) void off_rowscan_kernel(uint32_t *hist, uint32_t *tot,
                                                                  int64_t nblk)
{
    __shared__ uint32_t red[kRowThreads / kWave];
    const int tid = threadIdx.x, lane = lane_id(), wave = wave_id();
    uint32_t *row = hist + (int64_t)blockIdx.x * nblk;
    const uint32_t v = tid < nblk ? row[tid] : 0u;
    const uint32_t incl = wave_scan(v, 0u, AddOp{});
    if (lane == kWave - 1) red[wave] = incl;
    __syncthreads();
    uint32_t ex = incl - v, all = 0;
#pragma unroll
    for (int w = 0; w < kRowThreads / kWave; ++w) {
        if (w < wave) ex += red[w];
        all += red[w];
    }
    if (tid < nblk) row[tid] = ex;
    if (tid == 0) tot[blockIdx.x] = all;
}

__global__ __launch_bounds__(kOffThreads) void off_scatter_kernel(const int32_t *__restrict__ anc,
                                                                  int64_t P,
                                                                  const uint32_t *__restrict__ pos,
                                                                  const uint32_t *__restrict__ tot,
                                                                  uint32_t *__restrict__ bstart,
                                                                  int32_t *__restrict__ grouped,
                                                                  int bits, int64_t nb,
                                                                  int64_t nblk, int64_t per)
{
    __shared__ uint32_t cur[kMaxBuckets];     // next grouped position of each bucket
    __shared__ uint32_t cnt[kMaxBuckets];     // this chunk's count of each bucket
    __shared__ uint32_t lstart[kMaxBuckets];  // and its start in the staged chunk
    __shared__ int32_t stage[kBlockGrain];    // the chunk's ancestors by bucket
    __shared__ uint32_t red[kOffWaves];
    const int tid = threadIdx.x;
    // bucket tid starts after the smaller buckets, then after its ancestors
    // in the blocks before this one
    const uint32_t start = bucket_excl(tid < nb ? tot[tid] : 0u, red);
    if (tid < nb) {
        cur[tid] = start + pos[(int64_t)tid * nblk + blockIdx.x];
        cnt[tid] = 0;
        if (blockIdx.x == 0) bstart[tid] = start;  // for the count kernel
    }
    __syncthreads();
    const int64_t i0 = (int64_t)blockIdx.x * per, i1 = min(P, i0 + per);
    // chunks of kBlockGrain ancestors, four per thread: ranked inside their
    // bucket (LDS atomics), staged by bucket, then each bucket's run written
    // out contiguously
    for (int64_t c0 = i0; c0 < i1; c0 += kBlockGrain) {
        const int64_t c1 = min(i1, c0 + kBlockGrain);
        int32_t a[4];
        uint32_t rank[4];
        load_anc4(anc, c0 + 4 * (int64_t)tid, c1, a);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if (a[k] < 0 || (int64_t)a[k] >= P) a[k] = -1;  // past the chunk, or out of range
            rank[k] = a[k] >= 0 ? atomicAdd(&cnt[a[k] >> bits], 1u) : 0u;
        }
        __syncthreads();  // every rank taken before the counts are read
        const uint32_t ls = bucket_excl(tid < nb ? cnt[tid] : 0u, red);  // ends with a barrier
        if (tid < nb) lstart[tid] = ls;
        __syncthreads();
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (a[k] >= 0) stage[lstart[a[k] >> bits] + rank[k]] = a[k];
        __syncthreads();
        const uint32_t staged = lstart[nb - 1] + cnt[nb - 1];
        for (uint32_t q = tid; q < staged; q += kOffThreads) {
            const int32_t v = stage[q];
            const uint32_t b = (uint32_t)v >> bits;
            grouped[cur[b] + (q - lstart[b])] = v;
        }
        __syncthreads();
        if (tid < nb) {
            cur[tid] += cnt[tid];
            cnt[tid] = 0;
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(kOffThreads) void off_count_kernel(const int32_t *__restrict__ grouped,
                                                                int32_t *__restrict__ off,
                                                                int64_t P,
                                                                const uint32_t *__restrict__ tot,
                                                                const uint32_t *__restrict__ bstart,
                                                                int bits)
{
    extern __shared__ uint32_t c[];  // 2^bits counters
    const int tid = threadIdx.x, lane = lane_id();
    const int64_t bucket = int64_t(1) << bits;
    const int64_t b = blockIdx.x, jbase = b * bucket;
    const int64_t s = bstart[b], e = s + tot[b];  // this bucket's range of the grouped array
    for (int64_t r = tid; r < bucket; r += kOffThreads) c[r] = 0;
    __syncthreads();
    const uint64_t below = (1ull << lane) - 1ull;
    // whole waves run every round (the ballots below need them)
    for (int64_t q0 = s; q0 < e; q0 += kOffThreads) {
        const int64_t q = q0 + tid;
        const bool valid = q < e;
        const uint32_t key = valid ? (uint32_t)(grouped[q] - jbase) : 0u;
        // the lanes of this wave holding the same particle
        uint64_t peers = __ballot(valid);
        for (int bit = 0; bit < bits; ++bit) {  // uniform trip count
            const bool on = (key >> bit) & 1u;
            const uint64_t m = __ballot(on);
            peers &= on ? m : ~m;
        }
        if (valid && (peers & below) == 0) atomicAdd(&c[key], (uint32_t)__popcll(peers));
    }
    __syncthreads();
    const int64_t m = min(bucket, P - jbase);
    for (int64_t r = tid; r < m; r += kOffThreads) off[jbase + r] = (int32_t)c[r];
}

}  // namespace

size_t offspring_workspace_bytes(int64_t P)
{
    if (P < 1 || P > kMaxP) return 0;
    return off_layout(P).total;
}

int launch_offspring_ws(const int32_t *anc, int32_t *off, int64_t P, void *ws, int32_t *status,
                        hipStream_t stream)
{
    if (P > kMaxP) return launch_offspring(anc, off, P, status, stream);
    const OffLayout L = off_layout(P);
    char *w = static_cast<char *>(ws);
    uint32_t *hist = reinterpret_cast<uint32_t *>(w + L.hist);
    uint32_t *tot = reinterpret_cast<uint32_t *>(w + L.tot);
    uint32_t *bstart = reinterpret_cast<uint32_t *>(w + L.bstart);
    int32_t *grouped = reinterpret_cast<int32_t *>(w + L.grouped);
    const size_t smem = (size_t(1) << L.bits) * sizeof(uint32_t);
    if (allow_dynamic_lds(reinterpret_cast<const void *>(&off_count_kernel), smem)) return -3;
    const dim3 tb(kOffThreads);
    hipLaunchKernelGGL(off_hist_kernel, dim3((uint32_t)L.nblk), tb, 0, stream, anc, P, hist, L.bits,
                       L.nb, L.nblk, L.per, status);
    hipLaunchKernelGGL(off_rowscan_kernel, dim3((uint32_t)L.nb), dim3(kRowThreads), 0, stream, hist,
                       tot, L.nblk);
    hipLaunchKernelGGL(off_scatter_kernel, dim3((uint32_t)L.nblk), tb, 0, stream, anc, P, hist, tot,
                       bstart, grouped, L.bits, L.nb, L.nblk, L.per);
    hipLaunchKernelGGL(off_count_kernel, dim3((uint32_t)L.nb), tb, smem, stream, grouped, off, P,
                       tot, bstart, L.bits);
    return launch_status();
}

}  // namespace rs
