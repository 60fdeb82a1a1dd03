// Sorted-weight variants of the prefix-sum resamplers (Sec. 3 of the paper:
// the weights are sorted before the prefix sum, which shortens the
// multinomial bisection; the paper finds the sort costs more than it saves).
//
// Steps: the log-weights become sort keys (-0 as +0, so equal weights keep
// index order like any stable sort); a stable descending radix sort
// (rocPRIM) carries the particle indices along; the chosen resampler runs on
// the sorted weights; ancestors are mapped back through the permutation.
// Flagged inputs give identity ancestors, as the plain resamplers do.
#include <hip/hip_runtime.h>

#include <rocprim/device/device_radix_sort.hpp>

#include "launch.h"
#include "prefix.h"

namespace rs {
namespace {

constexpr int kThreads = 256;

__global__ __launch_bounds__(kThreads) void sort_keys_kernel(const float *__restrict__ lw,
                                                             float *__restrict__ keys,
                                                             int32_t *__restrict__ idx, int64_t P)
{
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < P; i += stride) {
        const float v = lw[i];
        keys[i] = v == 0.0f ? 0.0f : v;
        idx[i] = (int32_t)i;
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
    L.temp_bytes = al(16 * p + ((size_t)4 << 20));  // bound on the sort's scratch
    L.total = L.temp + L.temp_bytes;
    return L;
}

int launch_sorted(int kind, const float *lw, int32_t *anc, int64_t P, uint64_t seed,
                  uint32_t instance, void *ws, int32_t *status, hipStream_t stream)
{
    const SortedLayout L = sorted_layout(P, kind);
    char *w = static_cast<char *>(ws);
    float *keys_in = reinterpret_cast<float *>(w + L.keys_in);
    float *keys_out = reinterpret_cast<float *>(w + L.keys_out);
    int32_t *idx_in = reinterpret_cast<int32_t *>(w + L.idx_in);
    int32_t *perm = reinterpret_cast<int32_t *>(w + L.perm);
    int32_t *a_sorted = reinterpret_cast<int32_t *>(w + L.a_sorted);
    size_t need = 0;
    hipError_t e = rocprim::radix_sort_pairs_desc(nullptr, need, keys_in, keys_out, idx_in, perm,
                                                  (size_t)P, 0, 32, stream);
    if (e != hipSuccess) return record_hip_error(e);
    if (need > L.temp_bytes) return -2;
    hipLaunchKernelGGL(sort_keys_kernel, dim3(grid_for(P)), dim3(kThreads), 0, stream, lw, keys_in,
                       idx_in, P);
    size_t have = L.temp_bytes;
    e = rocprim::radix_sort_pairs_desc(w + L.temp, have, keys_in, keys_out, idx_in, perm,
                                       (size_t)P, 0, 32, stream);
    if (e != hipSuccess) return record_hip_error(e);
    int rc = launch_prefix(kind, keys_out, a_sorted, nullptr, P, seed, instance, nullptr, w,
                           status, stream);
    if (rc) return rc;
    hipLaunchKernelGGL(map_back_kernel, dim3(grid_for(P)), dim3(kThreads), 0, stream, a_sorted,
                       perm, anc, P, reinterpret_cast<const WsHeader *>(w));
    return launch_status();
}

}  // namespace rs
