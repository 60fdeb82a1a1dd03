// Offspring counts and the ancestor-indexed state copy (Sec. 2 of the paper:
// o_j is the number of offspring of particle j, a_i the ancestor of particle
// i; the copy carries the chosen ancestors' state to the next time step).
//
// Both are HBM-bound streams. The copy reads anc once, gathers rows of D
// binary32 values (16-byte vectors when D is a multiple of 4) and writes
// x_out fully coalesced. Offspring counting compresses equal neighbours
// inside a wave before its atomics, so sorted ancestors (stratified,
// systematic) cost about one atomic per distinct ancestor and unsorted ones
// (Metropolis, multinomial) one per particle.
#include <hip/hip_runtime.h>

#include "common.h"
#include "launch.h"

namespace rs {
namespace {

constexpr int kThreads = 256;

__global__ __launch_bounds__(kThreads) void zero_kernel(uint8_t *p, size_t bytes)
{
    const size_t stride = (size_t)gridDim.x * kThreads;
    const size_t n16 = (((uintptr_t)p & 15) == 0) ? bytes / 16 : 0;
    for (size_t q = (size_t)blockIdx.x * kThreads + threadIdx.x; q < n16; q += stride)
        reinterpret_cast<int4 *>(p)[q] = make_int4(0, 0, 0, 0);
    for (size_t b = 16 * n16 + (size_t)blockIdx.x * kThreads + threadIdx.x; b < bytes; b += stride)
        p[b] = 0;
}

__global__ __launch_bounds__(kThreads) void offspring_kernel(const int32_t *__restrict__ anc,
                                                             int32_t *__restrict__ off, int64_t P,
                                                             int32_t *status)
{
    const int lane = lane_id();
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    int fl = 0;
    // the loop bound is uniform per block, so whole waves run each ballot
    for (int64_t base = (int64_t)blockIdx.x * kThreads; base < P; base += stride) {
        const int64_t i = base + threadIdx.x;
        const bool in = i < P;
        const int32_t a = in ? anc[i] : -1;
        const bool ok = in && a >= 0 && (int64_t)a < P;
        if (in && !ok) fl |= kFlagBadAncestor;
        const int32_t prev = __shfl_up(a, 1, kWave);
        const bool prev_ok = __shfl_up((int)ok, 1, kWave) != 0;
        const bool head = ok && (lane == 0 || !prev_ok || prev != a);
        const uint64_t heads = __ballot(head);
        const uint64_t breaks = heads | __ballot(!ok);
        if (head) {
            const uint64_t above = breaks & ~((2ull << lane) - 1ull);
            const int next = above ? (__ffsll((long long)above) - 1) : kWave;
            atomicAdd(&off[a], next - lane);
        }
    }
    raise_flags(status, fl);
}

// Rows of D = 4 cols floats as 16-byte vectors. Each thread moves kRows
// rows spaced a grid apart, so its ancestor loads and row gathers are
// independent and in flight together, and every load/store instruction is
// coalesced across the wave (consecutive lanes, consecutive rows).
constexpr int kRows = 4;

__global__ __launch_bounds__(kThreads) void copy_rows_vec4(const int32_t *__restrict__ anc,
                                                           const float4 *__restrict__ x_in,
                                                           float4 *__restrict__ x_out, int64_t P,
                                                           int32_t cols, int32_t *status)
{
    const int64_t nthreads = (int64_t)gridDim.x * kThreads;
    int fl = 0;
    for (int64_t r0 = (int64_t)blockIdx.x * kThreads + threadIdx.x; r0 < P; r0 += kRows * nthreads) {
        int32_t a[kRows];
#pragma unroll
        for (int k = 0; k < kRows; ++k) {
            const int64_t r = r0 + k * nthreads;
            a[k] = r < P ? anc[r] : 0;
        }
        for (int32_t c = 0; c < cols; ++c) {
            float4 v[kRows];
#pragma unroll
            for (int k = 0; k < kRows; ++k) {
                const int64_t r = r0 + k * nthreads;
                const bool ok = a[k] >= 0 && (int64_t)a[k] < P;
                v[k] = (r < P && ok) ? x_in[(int64_t)a[k] * cols + c] : make_float4(0.f, 0.f, 0.f, 0.f);
                if (r < P && !ok) fl |= kFlagBadAncestor;
            }
#pragma unroll
            for (int k = 0; k < kRows; ++k) {
                const int64_t r = r0 + k * nthreads;
                if (r < P) x_out[r * cols + c] = v[k];
            }
        }
    }
    raise_flags(status, fl);
}

// Rows of COLS 16-byte vectors (D = 4 COLS, COLS = 2, 4 or 8): COLS
// consecutive lanes share a row, one vector each, so every load instruction
// reads whole rows; a row scattered by random ancestors is then fetched once
// instead of once per vector. Each thread handles kRows (row, vector) pairs
// spaced a grid apart, all loads in flight together.
template <int COLS>
__global__ __launch_bounds__(kThreads) void copy_rows_wide(const int32_t *__restrict__ anc,
                                                           const float4 *__restrict__ x_in,
                                                           float4 *__restrict__ x_out, int64_t P,
                                                           int32_t *status)
{
    const int64_t nthreads = (int64_t)gridDim.x * kThreads, total = P * COLS;
    int fl = 0;
    for (int64_t e0 = (int64_t)blockIdx.x * kThreads + threadIdx.x; e0 < total;
         e0 += kRows * nthreads) {
        int32_t a[kRows];
#pragma unroll
        for (int k = 0; k < kRows; ++k) {
            const int64_t e = e0 + k * nthreads;
            a[k] = e < total ? anc[e / COLS] : 0;
        }
        float4 v[kRows];
#pragma unroll
        for (int k = 0; k < kRows; ++k) {
            const int64_t e = e0 + k * nthreads;
            const bool ok = a[k] >= 0 && (int64_t)a[k] < P;
            v[k] = (e < total && ok) ? x_in[(int64_t)a[k] * COLS + (e % COLS)]
                                     : make_float4(0.f, 0.f, 0.f, 0.f);
            if (e < total && !ok) fl |= kFlagBadAncestor;
        }
#pragma unroll
        for (int k = 0; k < kRows; ++k) {
            const int64_t e = e0 + k * nthreads;
            if (e < total) x_out[e] = v[k];
        }
    }
    raise_flags(status, fl);
}

// D = 1: four rows per thread (one 16-byte ancestor load, four 4-byte
// gathers, one 16-byte store).
__global__ __launch_bounds__(kThreads) void copy_rows_d1(const int32_t *__restrict__ anc,
                                                         const float *__restrict__ x_in,
                                                         float *__restrict__ x_out, int64_t P,
                                                         int32_t *status)
{
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    const bool aligned = ((((uintptr_t)anc) | ((uintptr_t)x_out)) & 15) == 0;
    int fl = 0;
    for (int64_t q = (int64_t)blockIdx.x * kThreads + threadIdx.x; 4 * q < P; q += stride) {
        const int64_t i0 = 4 * q;
        if (aligned && i0 + 3 < P) {
            const int4 a = reinterpret_cast<const int4 *>(anc)[q];
            const int32_t av[4] = {a.x, a.y, a.z, a.w};
            float v[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const bool ok = av[k] >= 0 && (int64_t)av[k] < P;
                v[k] = ok ? x_in[av[k]] : 0.0f;
                if (!ok) fl |= kFlagBadAncestor;
            }
            reinterpret_cast<float4 *>(x_out)[q] = make_float4(v[0], v[1], v[2], v[3]);
        } else {
            for (int64_t i = i0; i < min(P, i0 + 4); ++i) {
                const int32_t a = anc[i];
                const bool ok = a >= 0 && (int64_t)a < P;
                x_out[i] = ok ? x_in[a] : 0.0f;
                if (!ok) fl |= kFlagBadAncestor;
            }
        }
    }
    raise_flags(status, fl);
}

// General D: one thread per element.
__global__ __launch_bounds__(kThreads) void copy_rows_scalar(const int32_t *__restrict__ anc,
                                                             const float *__restrict__ x_in,
                                                             float *__restrict__ x_out, int64_t P,
                                                             int32_t D, int32_t *status)
{
    const int64_t total = P * (int64_t)D;
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    int fl = 0;
    for (int64_t q = (int64_t)blockIdx.x * kThreads + threadIdx.x; q < total; q += stride) {
        const int64_t i = q / D, d = q - i * D;
        const int32_t a = anc[i];
        const bool ok = a >= 0 && (int64_t)a < P;
        x_out[q] = ok ? x_in[(int64_t)a * D + d] : 0.0f;
        if (!ok) fl |= kFlagBadAncestor;
    }
    raise_flags(status, fl);
}

uint32_t grid_for(int64_t work)
{
    int64_t g = (work + kThreads - 1) / kThreads;
    if (g < 1) g = 1;
    if (g > 16384) g = 16384;
    return (uint32_t)g;
}

}  // namespace

int launch_zero(void *ptr, size_t bytes, hipStream_t stream)
{
    if (bytes == 0) return 0;
    hipLaunchKernelGGL(zero_kernel, dim3(grid_for((int64_t)(bytes / 16 + 1))), dim3(kThreads), 0,
                       stream, static_cast<uint8_t *>(ptr), bytes);
    return launch_status();
}

int launch_offspring(const int32_t *anc, int32_t *off, int64_t P, int32_t *status,
                     hipStream_t stream)
{
    int rc = launch_zero(off, (size_t)P * sizeof(int32_t), stream);
    if (rc) return rc;
    hipLaunchKernelGGL(offspring_kernel, dim3(grid_for(P)), dim3(kThreads), 0, stream, anc, off, P,
                       status);
    return launch_status();
}

int launch_permute_copy(const int32_t *anc, const float *x_in, float *x_out, int64_t P, int32_t D,
                        int32_t *status, hipStream_t stream)
{
    const bool vec_ok = (D % 4 == 0) && ((((uintptr_t)x_in) | ((uintptr_t)x_out)) & 15) == 0;
    if (D == 1) {
        hipLaunchKernelGGL(copy_rows_d1, dim3(grid_for((P + 3) / 4)), dim3(kThreads), 0, stream,
                           anc, x_in, x_out, P, status);
    } else if (vec_ok) {
        const int cols = D / 4;
        const bool wide = cols == 2 || cols == 4 || cols == 8;
        const int64_t units = wide ? P * cols : P;  // (row, vector) pairs or rows
        int64_t grid = (units + kThreads * kRows - 1) / (kThreads * kRows);
        if (grid < 1) grid = 1;
        if (grid > 65535) grid = 65535;
        const float4 *in4 = reinterpret_cast<const float4 *>(x_in);
        float4 *out4 = reinterpret_cast<float4 *>(x_out);
        if (cols == 2)
            hipLaunchKernelGGL(copy_rows_wide<2>, dim3((uint32_t)grid), dim3(kThreads), 0, stream,
                               anc, in4, out4, P, status);
        else if (cols == 4)
            hipLaunchKernelGGL(copy_rows_wide<4>, dim3((uint32_t)grid), dim3(kThreads), 0, stream,
                               anc, in4, out4, P, status);
        else if (cols == 8)
            hipLaunchKernelGGL(copy_rows_wide<8>, dim3((uint32_t)grid), dim3(kThreads), 0, stream,
                               anc, in4, out4, P, status);
        else
            hipLaunchKernelGGL(copy_rows_vec4, dim3((uint32_t)grid), dim3(kThreads), 0, stream,
                               anc, in4, out4, P, cols, status);
    } else {
        hipLaunchKernelGGL(copy_rows_scalar, dim3(grid_for(P * (int64_t)D)), dim3(kThreads), 0,
                           stream, anc, x_in, x_out, P, D, status);
    }
    return launch_status();
}

}  // namespace rs
