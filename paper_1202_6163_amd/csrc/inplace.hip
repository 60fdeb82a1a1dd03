// Minimal-copy state update from offspring counts on gfx950.
//
// Method (Sec. 2: a resampler's output as offspring o_j, the number of copies
// of particle j; after resampling every particle carries weight 1 / P, so the
// population is the multiset {x_j repeated o_j times} and its slot order is
// free). Rows with o_j >= 1 stay in their slots; slot i with o_i = 0 (a hole)
// takes one of the extra copies of the particles with o_j >= 2 (o_j - 1 each):
// the r-th hole in slot order takes the r-th extra in order of j. No source is
// a hole, so the rows move in place, and only the holes are written: 8D bytes
// per hole instead of 8D per particle for a full ancestor-indexed copy.
//
// Design on MI355X: three launches over 1024-particle tiles.
//  1. ip_count_kernel: per tile the number of holes, of extras, and whether a
//     count is negative (one read of the offspring).
//  2. ip_table_kernel (one block): exclusive prefixes of both over the tiles
//     (exact, integer) and the validity of the counts (sum P <=> holes =
//     extras).
//  3. ip_move_kernel: block t ranks its holes [H_t, H_t + h_t); those ranks are
//     the extras of a run of source tiles, found by a wave-wide search of the
//     extras prefix. For each source tile the block rebuilds the tile's
//     in-tile extras prefix in LDS and bisects it for each hole in range,
//     then writes every slot's particle and copies the hole rows (16-byte
//     vectors when the rows allow).
#include <hip/hip_runtime.h>

#include "common.h"
#include "launch.h"
#include "prefix.h"

namespace rs {
namespace {

constexpr int kIpThreads = kTileThreads;  // 4 particles per thread, kTile per block
constexpr int kIpWaves = kIpThreads / kWave;

struct alignas(256) IpHeader {
    int32_t valid;  // counts non-negative and summing to P
    int32_t pad;
    int64_t holes;
    int64_t extras;
};

struct IpLayout {
    size_t header, h, e, bad, hpre, epre, total;
};

__host__ __device__ inline IpLayout ip_layout(int64_t P)
{
    const size_t n = (size_t)num_tiles(P);
    IpLayout L;
    L.header = 0;
    L.h = ws_align(sizeof(IpHeader));
    L.e = L.h + ws_align(n * sizeof(int64_t));
    L.bad = L.e + ws_align(n * sizeof(int64_t));
    L.hpre = L.bad + ws_align(n * sizeof(int32_t));
    L.epre = L.hpre + ws_align(n * sizeof(int64_t));
    L.total = L.epre + ws_align((n + 1) * sizeof(int64_t));
    return L;
}

// Exclusive prefix over the block's threads and the block total (integers,
// so any association order gives the same result).
template <typename T>
__device__ inline T block_excl(T v, T *red, T *total)
{
    const int lane = lane_id(), wave = wave_id();
    const T incl = wave_scan(v, (T)0, AddOp{});
    const T excl = wave_shift_up(incl);
    if (lane == kWave - 1) red[wave] = incl;
    __syncthreads();
    T wp = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < kIpWaves; ++w) {
        if (w < wave) wp += red[w];
        tot += red[w];
    }
    __syncthreads();
    *total = tot;
    return wp + excl;
}

// The thread's four offspring counts of tile t; slots past P count as 1
// (neither a hole nor an extra).
__device__ __forceinline__ void load_counts(const int32_t *__restrict__ off, int64_t P, int64_t t,
                                            int32_t o[4])
{
    const int64_t base = t * kTile + 4 * (int64_t)threadIdx.x;
    if (base + 3 < P && (((uintptr_t)(off + base)) & 15) == 0) {
        const int4 q = *reinterpret_cast<const int4 *>(off + base);
        o[0] = q.x, o[1] = q.y, o[2] = q.z, o[3] = q.w;
    } else {
#pragma unroll
        for (int k = 0; k < 4; ++k) o[k] = base + k < P ? off[base + k] : 1;
    }
}

__global__ __launch_bounds__(kIpThreads) void ip_count_kernel(const int32_t *__restrict__ off,
                                                              int64_t P, char *ws)
{
    __shared__ int64_t red[kIpWaves];
    const IpLayout L = ip_layout(P);
    const int64_t t = blockIdx.x;
    int32_t o[4];
    load_counts(off, P, t, o);
    int64_t h = 0, e = 0, bad = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        h += o[k] == 0;
        e += o[k] > 1 ? (int64_t)o[k] - 1 : 0;
        bad |= o[k] < 0;
    }
    int64_t th, te, tb;
    block_excl(h, red, &th);
    block_excl(e, red, &te);
    block_excl(bad, red, &tb);
    if (threadIdx.x == 0) {
        reinterpret_cast<int64_t *>(ws + L.h)[t] = th;
        reinterpret_cast<int64_t *>(ws + L.e)[t] = te;
        reinterpret_cast<int32_t *>(ws + L.bad)[t] = tb != 0;
    }
}

__global__ __launch_bounds__(kIpThreads) void ip_table_kernel(int64_t P, char *ws)
{
    __shared__ int64_t red[kIpWaves];
    const IpLayout L = ip_layout(P);
    const int64_t n = num_tiles(P);
    const int64_t *h = reinterpret_cast<const int64_t *>(ws + L.h);
    const int64_t *e = reinterpret_cast<const int64_t *>(ws + L.e);
    const int32_t *bad = reinterpret_cast<const int32_t *>(ws + L.bad);
    int64_t *hpre = reinterpret_cast<int64_t *>(ws + L.hpre);
    int64_t *epre = reinterpret_cast<int64_t *>(ws + L.epre);
    const int64_t per = (n + kIpThreads - 1) / kIpThreads;
    const int64_t t0 = min(n, (int64_t)threadIdx.x * per), t1 = min(n, t0 + per);
    int64_t sh = 0, se = 0, sb = 0;
    for (int64_t t = t0; t < t1; ++t) {
        sh += h[t];
        se += e[t];
        sb |= bad[t];
    }
    int64_t H, E, anybad;
    int64_t ph = block_excl(sh, red, &H);
    int64_t pe = block_excl(se, red, &E);
    block_excl(sb, red, &anybad);
    for (int64_t t = t0; t < t1; ++t) {
        hpre[t] = ph;
        epre[t] = pe;
        ph += h[t];
        pe += e[t];
    }
    if (threadIdx.x == 0) {
        epre[n] = E;
        IpHeader *hd = reinterpret_cast<IpHeader *>(ws + L.header);
        hd->valid = (anybad == 0 && H == E) ? 1 : 0;
        hd->holes = H;
        hd->extras = E;
    }
}

// First tile s in [0, n) whose extras range [epre[s], epre[s + 1]) contains
// rank r (r < epre[n]): the smallest s with epre[s + 1] > r. Wave 0 samples 64
// positions per round, so a round narrows the range 64-fold.
__device__ int64_t first_source_tile(const int64_t *epre, int64_t n, int64_t r)
{
    int64_t lo = 0, hi = n - 1;  // answer in [lo, hi]
    const int lane = lane_id();
    while (lo < hi) {
        const int64_t span = hi - lo + 1;
        const int64_t pos = lo + (span * lane) / kWave;  // non-decreasing over lanes, pos <= hi
        const bool above = epre[pos + 1] > r;
        const uint64_t mask = __ballot(above);
        int64_t nlo = lo, nhi = hi;
        if (mask) {
            const int f = __builtin_ctzll(mask);  // first sampled position with the property
            nhi = __shfl(pos, f);
            if (f > 0) nlo = __shfl(pos, f - 1) + 1;
        } else {
            nlo = __shfl(pos, kWave - 1) + 1;
        }
        lo = nlo;
        hi = nhi;
    }
    return lo;
}

__global__ __launch_bounds__(kIpThreads) void ip_move_kernel(const int32_t *__restrict__ off,
                                                             float *x, int64_t P, int32_t D,
                                                             int32_t *anc, const char *ws,
                                                             int32_t *status)
{
    __shared__ int32_t red[kIpWaves];
    __shared__ int32_t incl[kTile];     // a source tile's inclusive extras prefix
    __shared__ int32_t sh_hole[kTile];  // the block's holes by rank: slot
    __shared__ int32_t sh_src[kTile];   // and source particle
    __shared__ int64_t sh_s0;
    const IpLayout L = ip_layout(P);
    const IpHeader *hd = reinterpret_cast<const IpHeader *>(ws + L.header);
    const int64_t *epre = reinterpret_cast<const int64_t *>(ws + L.epre);
    const int64_t n = num_tiles(P), t = blockIdx.x, base = t * kTile;
    const int tid = threadIdx.x;
    const int64_t j0 = base + 4 * (int64_t)tid;

    int32_t o[4];
    load_counts(off, P, t, o);
    const bool valid = hd->valid != 0;
    if (!valid) {  // the counts are not a resampling: the state stays, identity slots
        if (t == 0 && tid == 0) raise_flags(status, kFlagBadAncestor);
        if (anc)
            for (int k = 0; k < 4; ++k)
                if (j0 + k < P) anc[j0 + k] = (int32_t)(j0 + k);
        return;
    }
    // ranks of this tile's holes
    int32_t nh = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) nh += o[k] == 0;
    int32_t ht;
    const int32_t q0 = block_excl(nh, red, &ht);
    int32_t rank[4];
    {
        int32_t q = q0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            rank[k] = -1;
            if (o[k] == 0) {
                rank[k] = q;
                sh_hole[q] = (int32_t)(j0 + k);
                sh_src[q] = -1;
                ++q;
            }
        }
    }
    if (ht > 0) {
        const int64_t R0 = reinterpret_cast<const int64_t *>(ws + L.hpre)[t], R1 = R0 + ht;
        if (tid < kWave) {
            const int64_t s0 = first_source_tile(epre, n, R0);
            if (tid == 0) sh_s0 = s0;
        }
        __syncthreads();
        for (int64_t s = sh_s0; s < n; ++s) {  // uniform
            const int64_t Es = epre[s], Es1 = epre[s + 1];
            if (Es >= R1) break;
            if (Es1 == Es) continue;
            int32_t o2[4];
            load_counts(off, P, s, o2);
            int32_t ex[4], sum = 0;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                ex[k] = o2[k] > 1 ? o2[k] - 1 : 0;
                sum += ex[k];
            }
            int32_t tot;
            int32_t run = block_excl(sum, red, &tot);  // ends with a barrier
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                run += ex[k];
                incl[4 * tid + k] = run;
            }
            __syncthreads();
            // the block's holes whose ranks fall in this tile's extras
            const int64_t qa = max(Es - R0, (int64_t)0), qb = min(Es1 - R0, (int64_t)ht);
            for (int64_t q = qa + tid; q < qb; q += kIpThreads) {
                const int32_t loc = (int32_t)(R0 + q - Es);
                int j = 0;  // first j with incl[j] > loc
#pragma unroll
                for (int step = kTile / 2; step >= 1; step >>= 1)
                    if (incl[j + step - 1] <= loc) j += step;
                sh_src[q] = (int32_t)(s * kTile + j);
            }
            __syncthreads();  // incl is rebuilt for the next tile
        }
    }
    __syncthreads();
    int fl = 0;
    if (anc) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if (j0 + k >= P) continue;
            int32_t a = (int32_t)(j0 + k);
            if (rank[k] >= 0) {
                a = sh_src[rank[k]];
                if (a < 0) fl |= kFlagInternal;
            }
            anc[j0 + k] = a;
        }
    }
    // the hole rows, copied by the whole block
    const bool vec = (D % 4 == 0) && ((((uintptr_t)x) & 15) == 0);
    if (vec) {
        const int cols = D / 4;
        float4 *x4 = reinterpret_cast<float4 *>(x);
        for (int64_t e = tid; e < (int64_t)ht * cols; e += kIpThreads) {
            const int64_t q = e / cols, c = e - q * cols;
            const int32_t src = sh_src[q];
            if (src < 0) {  // a hole left without a source: a library bug
                fl |= kFlagInternal;
                continue;
            }
            x4[(int64_t)sh_hole[q] * cols + c] = x4[(int64_t)src * cols + c];
        }
    } else {
        for (int64_t e = tid; e < (int64_t)ht * D; e += kIpThreads) {
            const int64_t q = e / D, d = e - q * D;
            const int32_t src = sh_src[q];
            if (src < 0) {
                fl |= kFlagInternal;
                continue;
            }
            x[(int64_t)sh_hole[q] * D + d] = x[(int64_t)src * D + d];
        }
    }
    raise_flags(status, fl);
}

}  // namespace

size_t inplace_workspace_bytes(int64_t P) { return ip_layout(P).total; }

int launch_offspring_update_inplace(const int32_t *off, float *x, int64_t P, int32_t D,
                                    int32_t *anc, void *ws, int32_t *status, hipStream_t stream)
{
    char *w = static_cast<char *>(ws);
    const dim3 grid((uint32_t)num_tiles(P)), tb(kIpThreads);
    hipLaunchKernelGGL(ip_count_kernel, grid, tb, 0, stream, off, P, w);
    hipLaunchKernelGGL(ip_table_kernel, dim3(1), tb, 0, stream, P, w);
    hipLaunchKernelGGL(ip_move_kernel, grid, tb, 0, stream, off, x, P, D, anc, w, status);
    return launch_status();
}

}  // namespace rs
