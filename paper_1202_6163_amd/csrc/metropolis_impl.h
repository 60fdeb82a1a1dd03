// Device pieces of the Metropolis resampler shared by the single-call kernel
// (metropolis.hip) and the batched persistent kernel (batch.hip): the exact
// acceptance test and the per-chain loop. See metropolis.hip for the method.
#pragma once

#include <hip/hip_runtime.h>

#include "common.h"

namespace rs {
namespace mh {

constexpr float kLn2 = 0.693147180559945309417f;
constexpr float kFastMargin = 0x1p-16f;

__device__ __forceinline__ float approx_log_u(float u)
{
    return __builtin_amdgcn_logf(u) * kLn2;
}

// Exact decision of L(u) < d, L the correctly rounded binary32 log: a
// difference d >= 0 always accepts (L(u) < 0), NaN never does; otherwise
// the hardware log decides when d is farther than 2^-16 |log u| from it and
// the binary64 log decides the rest.
__device__ __forceinline__ bool accept_move(float d, float la, float u)
{
    if (!(d < 0.0f)) return d >= 0.0f;
    const float t = fabsf(la) * kFastMargin;
    if (la + t < d) return true;
    if (la - t >= d) return false;
    return exact_log_u(u) < d;
}

// The draws of iterations n0 .. n0 + UNROLL - 1 of chain i (n0 even): the
// proposals, their weights and the uniforms with their approximate logs.
template <int UNROLL>
__device__ __forceinline__ void draw_round(const float *w, uint32_t P, uint64_t seed,
                                           uint32_t instance, uint32_t i, uint32_t n0,
                                           uint32_t jj[UNROLL], float vv[UNROLL],
                                           float uu[UNROLL], float la[UNROLL])
{
#pragma unroll
    for (int p = 0; p < UNROLL / 2; ++p) {
        const Block4 b = philox(seed, i, instance, (n0 >> 1) + (uint32_t)p, kTagMetropolis);
        jj[2 * p] = uniform_index(b.r0, P);
        uu[2 * p] = grid_uniform(b.r1);
        jj[2 * p + 1] = uniform_index(b.r2, P);
        uu[2 * p + 1] = grid_uniform(b.r3);
    }
#pragma unroll
    for (int s = 0; s < UNROLL; ++s) {
        vv[s] = w[jj[s]];
        la[s] = approx_log_u(uu[s]);
    }
}

// Chain i on one lane: B iterations from k = i; returns the ancestor.
template <int UNROLL>
__device__ __forceinline__ uint32_t chain(const float *w, uint32_t P, uint32_t B, uint64_t seed,
                                          uint32_t instance, uint32_t i)
{
    uint32_t k = i;
    float lk = w[i];
    for (uint32_t n0 = 0; n0 < B; n0 += UNROLL) {
        uint32_t jj[UNROLL];
        float uu[UNROLL], vv[UNROLL], la[UNROLL];
        draw_round<UNROLL>(w, P, seed, instance, i, n0, jj, vv, uu, la);
#pragma unroll
        for (int s = 0; s < UNROLL; ++s) {
            if (n0 + s < B && accept_move(vv[s] - lk, la[s], uu[s])) {
                k = jj[s];
                lk = vv[s];
            }
        }
    }
    return k;
}

__device__ __forceinline__ int weight_flags(float v)
{
    if (isnan(v)) return kFlagNan;
    if (isinf(v) && v > 0.0f) return kFlagPosInf;
    return 0;
}

}  // namespace mh
}  // namespace rs
