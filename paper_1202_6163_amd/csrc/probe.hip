// Measurement probes: device ceilings the Metropolis kernel is compared with.
// Not part of any resampler.
//  - gather probe: random 4-byte loads from an n-float array (the Metropolis
//    proposal gathers without the chains' arithmetic);
//  - Philox probe: Philox4x32-10 blocks alone (the chains' random numbers
//    without their gathers).
// Each thread folds what it loads or draws into one word so the compiler
// keeps the work, and writes that word once.
#include <hip/hip_runtime.h>

#include "common.h"
#include "launch.h"

namespace rs {
namespace {

constexpr int kThreads = 256;
constexpr int kPerRound = 8;  // independent loads / blocks in flight per thread

__global__ __launch_bounds__(kThreads) void gather_probe_kernel(const float *__restrict__ w,
                                                                uint32_t n, uint32_t rounds,
                                                                uint32_t salt, float *out)
{
    const uint32_t tid = blockIdx.x * kThreads + threadIdx.x;
    uint32_t x = tid * 0x9E3779B9u + salt;
    float acc = 0.0f;
    for (uint32_t r = 0; r < rounds; ++r) {
        float v[kPerRound];
#pragma unroll
        for (int k = 0; k < kPerRound; ++k) {
            x ^= x << 13;  // xorshift32: a cheap index stream
            x ^= x >> 17;
            x ^= x << 5;
            v[k] = w[uniform_index(x, n)];
        }
#pragma unroll
        for (int k = 0; k < kPerRound; ++k) acc += v[k];
    }
    out[tid] = acc;
}

__global__ __launch_bounds__(kThreads) void philox_probe_kernel(uint64_t seed, uint32_t rounds,
                                                                uint32_t *out)
{
    const uint32_t tid = blockIdx.x * kThreads + threadIdx.x;
    uint32_t acc = 0;
    for (uint32_t r = 0; r < rounds; ++r) {
#pragma unroll
        for (int k = 0; k < kPerRound / 2; ++k) {
            const Block4 b = philox(seed, tid, r, (uint32_t)k, 9u);
            acc ^= b.r0 ^ b.r1 ^ b.r2 ^ b.r3;
        }
    }
    out[tid] = acc;
}

}  // namespace

int launch_gather_probe(const float *w, uint32_t n, uint32_t threads, uint32_t rounds,
                        uint32_t salt, float *out, hipStream_t stream)
{
    hipLaunchKernelGGL(gather_probe_kernel, dim3(threads / kThreads), dim3(kThreads), 0, stream, w,
                       n, rounds, salt, out);
    return launch_status();
}

int launch_philox_probe(uint64_t seed, uint32_t threads, uint32_t rounds, uint32_t *out,
                        hipStream_t stream)
{
    hipLaunchKernelGGL(philox_probe_kernel, dim3(threads / kThreads), dim3(kThreads), 0, stream,
                       seed, rounds, out);
    return launch_status();
}

}  // namespace rs
