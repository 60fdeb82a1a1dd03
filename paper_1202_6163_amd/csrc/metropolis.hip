// Metropolis resampler on gfx950 (Sec. 2 of the paper: Fig. 1(d), the
// paragraph on the number of iterations B, and the convergence analysis,
// which fixes the proposal as uniform over all P indices).
//
// Chain i starts at k = i and runs B Metropolis steps on the weights: propose
// j uniformly, draw u, move iff log u < lw[j] - lw[k] (binary32 difference,
// correctly rounded binary32 log u). Only weight ratios are used, so chains
// never communicate and the whole resampling is one launch.
//
// Design on MI355X:
//  - Draws are counter-based (Philox block (i, instance, n/2, 1) feeds
//    iterations n and n+1), so a lane can generate every proposal and gather
//    every proposed weight of a chain before taking any decision: the
//    proposals and gathers do not depend on the chain state. Only the
//    accept/reject sequence is serial.
//  - Weights are staged in LDS when 4P bytes fit the tuned threshold;
//    otherwise proposals gather from L2 / the Infinity Cache.
//  - For small P the GPU has more lanes than chains: G lanes then share one
//    chain. Each lane generates UNROLL consecutive iterations' draws, gathers
//    and approximate logs in parallel, and the lanes then take their
//    decisions in iteration order, passing (k, lw[k]) down the group. The
//    decisions are the same as one lane's, bit for bit.
//  - log u: the hardware log2 approximation decides whenever the threshold is
//    farther than 2^-16 |log u| away (its error on the u grid is far smaller;
//    the test suite checks every grid point on the device); otherwise the
//    binary64 log decides. A difference d >= 0 always accepts (log u < 0)
//    and a NaN difference never does, with no log at all.
#include <hip/hip_runtime.h>

#include "common.h"
#include "launch.h"
#include "metropolis_impl.h"

namespace rs {
namespace {

using namespace mh;

template <int UNROLL, bool STAGE>
__global__ __launch_bounds__(1024) void metropolis_kernel(const float *__restrict__ lw,
                                                          int32_t *__restrict__ anc, uint32_t P,
                                                          uint32_t B, uint64_t seed,
                                                          uint32_t instance, int lpc_log2,
                                                          int32_t *status, const uint32_t *B_dev,
                                                          Rows rows)
{
    static_assert(UNROLL % 2 == 0, "one Philox block feeds two iterations");
    if (B_dev) B = min(B, *B_dev);  // iteration count computed on the device
    extern __shared__ float staged[];
    const float *w = lw;
    if (STAGE) {
        const bool aligned = (((uintptr_t)lw) & 15) == 0;
        const uint32_t P4 = aligned ? P / 4 : 0;
        for (uint32_t q = threadIdx.x; q < P4; q += blockDim.x)
            reinterpret_cast<float4 *>(staged)[q] = reinterpret_cast<const float4 *>(lw)[q];
        for (uint32_t i = 4 * P4 + threadIdx.x; i < P; i += blockDim.x) staged[i] = lw[i];
        __syncthreads();
        w = staged;
    }
    const uint32_t G = 1u << lpc_log2;
    const int src_base = lane_id() & ~(int)(G - 1);
    const uint64_t total = (uint64_t)P << lpc_log2;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t gt = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; gt < total; gt += stride) {
        const uint32_t i = (uint32_t)(gt >> lpc_log2);
        const uint32_t g = (uint32_t)(gt & (G - 1));
        if (g == 0) raise_flags(status, weight_flags(w[i]));
        if (G == 1) {
            const uint32_t a = chain<UNROLL>(w, P, B, seed, instance, i);
            anc[i] = (int32_t)a;
            if (rows.x_in) copy_row(rows, i, a, 0, 1);
            continue;
        }
        uint32_t k = i;
        float lk = w[i];
        for (uint32_t r0 = 0; r0 < B; r0 += G * UNROLL) {
            const uint32_t n0 = r0 + g * UNROLL;  // even
            uint32_t jj[UNROLL];
            float uu[UNROLL], vv[UNROLL], la[UNROLL];
            draw_round<UNROLL>(w, P, seed, instance, i, n0, jj, vv, uu, la);
            // decisions in iteration order: lane gg of the group, then the next
            for (uint32_t gg = 0; gg < G; ++gg) {
                if (g == gg) {
#pragma unroll
                    for (int s = 0; s < UNROLL; ++s) {
                        if (n0 + s < B && accept_move(vv[s] - lk, la[s], uu[s])) {
                            k = jj[s];
                            lk = vv[s];
                        }
                    }
                }
                k = (uint32_t)__shfl((int)k, src_base + (int)gg, kWave);
                lk = __shfl(lk, src_base + (int)gg, kWave);
            }
        }
        if (g == 0) anc[i] = (int32_t)k;
        if (rows.x_in) copy_row(rows, i, k, (int)g, (int)G);  // the group shares the row
    }
}

template <int UNROLL, bool STAGE>
int launch_variant(const float *lw, int32_t *anc, uint32_t P, uint32_t B, uint64_t seed,
                   uint32_t instance, int lpc_log2, int block, int32_t *status,
                   const uint32_t *B_dev, const Rows &rows, hipStream_t stream)
{
    const uint64_t threads = (uint64_t)P << lpc_log2;
    uint64_t grid = (threads + block - 1) / block;
    if (grid > (1u << 20)) grid = 1u << 20;
    size_t smem = 0;
    if (STAGE) {
        smem = (size_t)P * sizeof(float);
        if (allow_dynamic_lds(reinterpret_cast<const void *>(&metropolis_kernel<UNROLL, STAGE>),
                              smem))
            return -3;
    }
    hipLaunchKernelGGL((metropolis_kernel<UNROLL, STAGE>), dim3((uint32_t)grid), dim3(block),
                       smem, stream, lw, anc, P, B, seed, instance, lpc_log2, status, B_dev, rows);
    return launch_status();
}

// Lanes per chain when not fixed by the tuning: up to 2^16 threads in all,
// no more lanes than the iterations can use, and never two (measured at
// unroll 4, block 256: a two-lane group was slower than both one lane and
// four at every P from 4096 to 262144; past 2^16 threads the extra lanes
// only add group shuffles, e.g. P = 65536, B = 64: 20.0 us with one lane,
// 27.0 with two, 28.4 with four).
int auto_lanes_log2(uint32_t P, uint32_t B, int unroll)
{
    const uint64_t target = 1u << 16;
    int lg = 0;
    while (lg < 6 && ((uint64_t)P << (lg + 1)) <= target && ((uint64_t)unroll << (lg + 1)) <= B)
        ++lg;
    return lg == 1 ? 0 : lg;
}

// Both logs of every point of the u grid (m = 0 .. 2^23 - 1, u = (2m+1) 2^-24).
__global__ __launch_bounds__(256) void log_u_table_kernel(float *approx, float *exact)
{
    const uint32_t m = blockIdx.x * 256u + threadIdx.x;
    if (m >= (1u << 23)) return;
    const float u = grid_uniform(m << 9);
    if (approx) approx[m] = approx_log_u(u);
    if (exact) exact[m] = exact_log_u(u);
}

}  // namespace

int launch_log_u_table(float *approx, float *exact, hipStream_t stream)
{
    hipLaunchKernelGGL(log_u_table_kernel, dim3((1u << 23) / 256), dim3(256), 0, stream, approx,
                       exact);
    return launch_status();
}

int launch_metropolis_dev_B(const float *lw, int32_t *anc, int64_t P, uint32_t B,
                            const uint32_t *B_dev, uint64_t seed, uint32_t instance,
                            int32_t *status, const MetropolisTuning &tune, hipStream_t stream,
                            const Rows &rows)
{
    const uint32_t p = (uint32_t)P;
    int lg = 0;
    if (tune.lanes_per_chain > 0) {
        while ((1 << lg) < tune.lanes_per_chain) ++lg;
    } else {
        lg = auto_lanes_log2(p, B, tune.unroll);
    }
    int max_smem = 0, dev = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&max_smem, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
    const bool stage = P <= tune.lds_max_p && (int64_t)P * (int64_t)sizeof(float) <= max_smem;
    const int blk = tune.block;
#define RS_METRO_CASE(U)                                                                       \
    case U:                                                                                    \
        return stage ? launch_variant<U, true>(lw, anc, p, B, seed, instance, lg, blk, status, \
                                               B_dev, rows, stream)                            \
                     : launch_variant<U, false>(lw, anc, p, B, seed, instance, lg, blk,        \
                                                status, B_dev, rows, stream);
    switch (tune.unroll) {
        RS_METRO_CASE(2)
        RS_METRO_CASE(4)
        RS_METRO_CASE(8)
        RS_METRO_CASE(16)
    default:
        return -1;
    }
#undef RS_METRO_CASE
}

int launch_metropolis(const float *lw, int32_t *anc, int64_t P, uint32_t B, uint64_t seed,
                      uint32_t instance, int32_t *status, const MetropolisTuning &tune,
                      hipStream_t stream, const Rows &rows)
{
    return launch_metropolis_dev_B(lw, anc, P, B, nullptr, seed, instance, status, tune, stream,
                                   rows);
}

int launch_metropolis_adaptive(const float *lw, int32_t *anc, int64_t P, double eps,
                               uint32_t B_max, uint64_t seed, uint32_t instance, void *ws,
                               uint32_t *B_used, int32_t *status, const MetropolisTuning &tune,
                               hipStream_t stream)
{
    const int rc = launch_adaptive_B(lw, P, eps, B_max, ws, B_used, status, stream);
    if (rc) return rc;
    return launch_metropolis_dev_B(lw, anc, P, B_max, adaptive_B_slot(ws), seed, instance, status,
                                   tune, stream);
}

}  // namespace rs
