// Number of Metropolis iterations from the paper's convergence analysis
// (Sec. 2, eqs. (1)-(5)), shared by the host helper and the device-side
// adaptive resampler so both compute the same B.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rs {

// Smallest integer B >= 0 with lambda^B <= eps (alpha + beta) / max(alpha, beta)
// for the two-state chain "sits at the heaviest particle": alpha =
// (1 - w_max) / (P w_max), beta = 1 / P, lambda = 1 - alpha - beta (eq. (4);
// eq. (5) solves it for 0 < lambda < 1; lambda = 0, uniform weights, needs
// one step). w_max is the largest normalised weight.
__host__ __device__ inline uint32_t iterations_for(int64_t P, double w_max, double eps)
{
    if (P < 2 || !(w_max > 0.0) || w_max > 1.0 || !(eps > 0.0)) return 0;
    const double beta = 1.0 / (double)P;
    const double alpha = (1.0 - w_max) / ((double)P * w_max);
    const double lambda = 1.0 - alpha - beta;
    const double rhs = eps * (alpha + beta) / fmax(alpha, beta);
    if (rhs >= 1.0) return 0;
    if (!(lambda > 0.0)) return 1;
    const double b = ceil(log(rhs) / log(lambda));
    if (!(b > 0.0)) return 0;
    if (b >= 4294967295.0) return 4294967295u;
    return (uint32_t)b;
}

}  // namespace rs
