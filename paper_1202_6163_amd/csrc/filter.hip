// Bootstrap particle filter steps around the resampler (Sec. 1 of the paper:
// initialisation, propagation, weighting; resampling is the library's other
// entry points). Model: x_0 ~ N(0, I), x_t = A x_{t-1} + N(0, q I),
// y_t = x_t + N(0, r I). The proposal is the transition, so the log-weight is
// the observation log-density.
//
// Gaussian noise: Box-Muller on Philox block (i, t, h, 5) for components
// 4h .. 4h+3: words (r0, r1) give components 4h, 4h+1 and (r2, r3) give
// 4h+2, 4h+3, with u1 = (r + 1/2) 2^-32, u2 = r' 2^-32,
// z = sqrt(-2 log u1) (cos, sin)(2 pi u2). Time 0 draws the initial state.
//
// One thread per particle; the D x D transition matrix sits in LDS; the
// matrix-vector product and the weight accumulate in binary64 and round to
// binary32 state once per component. Rows are read and written as 16-byte
// vectors when D is a multiple of 4.
//
// Batches of K filters (particle MCMC evaluates many parameter values at
// once): filter k owns rows [k P, (k+1) P), draws with Philox key seed + k and
// may have its own noise variance q_k, so it computes exactly what a single
// filter with key seed + k and variance q_k computes.
#include <hip/hip_runtime.h>

#include "common.h"
#include "launch.h"

namespace rs {
namespace {

constexpr int kFilterThreads = 256;
constexpr int kMaxD = 64;

// One Box-Muller pair from two Philox words.
__device__ __forceinline__ void box_muller(uint32_t ra, uint32_t rb, double *z0, double *z1)
{
    const double two_pi = 6.283185307179586476925286766559;
    const double u1 = ((double)ra + 0.5) * 0x1p-32;
    const double u2 = (double)rb * 0x1p-32;
    const double rad = sqrt(-2.0 * log(u1));
    double sn, cs;
    sincos(two_pi * u2, &sn, &cs);  // one argument reduction for both
    *z0 = rad * cs;
    *z1 = rad * sn;
}

__device__ __forceinline__ void normals(uint64_t seed, uint32_t i, uint32_t t, int D, double *z)
{
    for (int h = 0; 4 * h < D; ++h) {
        const Block4 b = philox(seed, i, t, (uint32_t)h, kTagFilterNoise);
        const uint32_t r[4] = {b.r0, b.r1, b.r2, b.r3};
#pragma unroll
        for (int pair = 0; pair < 2; ++pair) {
            double z0, z1;
            box_muller(r[2 * pair], r[2 * pair + 1], &z0, &z1);
            const int d0 = 4 * h + 2 * pair;
            if (d0 < D) z[d0] = z0;
            if (d0 + 1 < D) z[d0 + 1] = z1;
        }
    }
}

__global__ __launch_bounds__(kFilterThreads) void filter_init_kernel(float *__restrict__ x,
                                                                     int64_t P, int64_t K, int D,
                                                                     uint64_t seed)
{
    double z[kMaxD];
    for (int64_t g = blockIdx.x * (int64_t)kFilterThreads + threadIdx.x; g < K * P;
         g += (int64_t)gridDim.x * kFilterThreads) {
        const int64_t k = g / P, i = g - k * P;
        normals(seed + (uint64_t)k, (uint32_t)i, 0u, D, z);
        for (int d = 0; d < D; ++d) x[g * D + d] = (float)z[d];
    }
}

template <int DC>  // compile-time D (0 = runtime D)
__global__ __launch_bounds__(kFilterThreads) void propagate_weight_kernel(
    const float *__restrict__ x_in, float *__restrict__ x_out, float *__restrict__ lw, int64_t P,
    int64_t K, int Drt, const double *__restrict__ A, const float *__restrict__ y, double sq,
    const double *__restrict__ q_k, double r, double norm, uint64_t seed, uint32_t t)
{
    const int D = DC > 0 ? DC : Drt;
    __shared__ double sA[kMaxD * kMaxD];
    __shared__ double sy[kMaxD];
    for (int k = threadIdx.x; k < D * D; k += kFilterThreads) sA[k] = A[k];
    for (int k = threadIdx.x; k < D; k += kFilterThreads) sy[k] = (double)y[k];
    __syncthreads();
    double xv[DC > 0 ? DC : kMaxD];
    for (int64_t g = blockIdx.x * (int64_t)kFilterThreads + threadIdx.x; g < K * P;
         g += (int64_t)gridDim.x * kFilterThreads) {
        const int64_t k = g / P, i = g - k * P;
        const double sqk = q_k ? sqrt(q_k[k]) : sq;
        const float *xi = x_in + g * D;
        if (DC > 0 && DC % 4 == 0) {
#pragma unroll
            for (int q = 0; q < D / 4; ++q) {
                const float4 v = reinterpret_cast<const float4 *>(xi)[q];
                xv[4 * q] = v.x; xv[4 * q + 1] = v.y; xv[4 * q + 2] = v.z; xv[4 * q + 3] = v.w;
            }
        } else {
            for (int d = 0; d < D; ++d) xv[d] = (double)xi[d];
        }
        // each noise pair is drawn just before the two rows that use it, so
        // only two noise values are live (all D at once, with the inlined
        // binary64 log and sincos, took over 250 VGPRs: one wave per SIMD)
        double ss = 0.0;
        float out[DC > 0 ? DC : kMaxD];
        for (int h = 0; 4 * h < D; ++h) {
            const Block4 bl = philox(seed + (uint64_t)k, (uint32_t)i, t, (uint32_t)h,
                                     kTagFilterNoise);
            const uint32_t rw[4] = {bl.r0, bl.r1, bl.r2, bl.r3};
#pragma unroll
            for (int pair = 0; pair < 2; ++pair) {
                const int d0 = 4 * h + 2 * pair;
                if (d0 >= D) break;
                double zp[2];
                box_muller(rw[2 * pair], rw[2 * pair + 1], &zp[0], &zp[1]);
#pragma unroll
                for (int e = 0; e < 2; ++e) {
                    const int a = d0 + e;
                    if (a < D) {
                        double acc = 0.0;
                        for (int b = 0; b < D; ++b) acc += sA[a * D + b] * xv[b];
                        const float xa = (float)(acc + sqk * zp[e]);
                        out[a] = xa;
                        const double ev = sy[a] - (double)xa;
                        ss += ev * ev;
                    }
                }
            }
        }
        float *xo = x_out + g * D;
        if (DC > 0 && DC % 4 == 0) {
#pragma unroll
            for (int q = 0; q < D / 4; ++q)
                reinterpret_cast<float4 *>(xo)[q] =
                    make_float4(out[4 * q], out[4 * q + 1], out[4 * q + 2], out[4 * q + 3]);
        } else {
            for (int d = 0; d < D; ++d) xo[d] = out[d];
        }
        lw[g] = (float)(norm - 0.5 * ss / r);
    }
}

uint32_t filter_grid(int64_t P)
{
    int64_t g = (P + kFilterThreads - 1) / kFilterThreads;
    if (g < 1) g = 1;
    if (g > 65535) g = 65535;
    return (uint32_t)g;
}

// log Z-hat = sum_t (lse_t - log P), added term by term in time order (the
// order a sequential filter accumulates it in). One lane: T is small.
__global__ void filter_loglik_kernel(const double *__restrict__ lse, int32_t T, int64_t P,
                                     double *__restrict__ out)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const double log_p = log((double)P);
    double ll = 0.0;
    for (int32_t t = 0; t < T; ++t) ll += lse[t] - log_p;
    out[0] = ll;
}

}  // namespace

int launch_filter_loglik(const double *lse, int32_t T, int64_t P, double *out, hipStream_t stream)
{
    hipLaunchKernelGGL(filter_loglik_kernel, dim3(1), dim3(64), 0, stream, lse, T, P, out);
    return launch_status();
}

int launch_filter_init(float *x, int64_t P, int64_t K, int32_t D, uint64_t seed,
                       hipStream_t stream)
{
    hipLaunchKernelGGL(filter_init_kernel, dim3(filter_grid(K * P)), dim3(kFilterThreads), 0,
                       stream, x, P, K, (int)D, seed);
    return launch_status();
}

int launch_filter_step(const float *x_in, float *x_out, float *lw, int64_t P, int64_t K,
                       int32_t D, const double *A, const float *y, double q, const double *q_k,
                       double r, uint64_t seed, uint32_t t, hipStream_t stream)
{
    const double log_two_pi = 1.8378770664093454835606594728112;
    const double norm = -0.5 * (double)D * (log_two_pi + log(r));
    const double sq = sqrt(q);
    const bool vec = ((((uintptr_t)x_in) | ((uintptr_t)x_out)) & 15) == 0;
    const dim3 grid(filter_grid(K * P)), block(kFilterThreads);
#define RS_FILTER_LAUNCH(DC)                                                                       \
    hipLaunchKernelGGL(propagate_weight_kernel<DC>, grid, block, 0, stream, x_in, x_out, lw, P, K, \
                       (int)D, A, y, sq, q_k, r, norm, seed, t)
    if (D == 8 && vec) {
        RS_FILTER_LAUNCH(8);
    } else if (D == 4 && vec) {
        RS_FILTER_LAUNCH(4);
    } else {
        RS_FILTER_LAUNCH(0);
    }
#undef RS_FILTER_LAUNCH
    return launch_status();
}

}  // namespace rs
