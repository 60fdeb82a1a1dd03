// Internal launchers behind the C ABI (argument checking is done by the
// caller in capi.cpp; these only enqueue kernels). Return 0 or -3 (launch
// failure).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rs {

struct MetropolisTuning {
    int32_t block;
    int32_t unroll;
    int64_t lds_max_p;
    int32_t lanes_per_chain;  // 0: chosen from P and B
};

int launch_metropolis(const float *lw, int32_t *anc, int64_t P, uint32_t B, uint64_t seed,
                      uint32_t instance, int32_t *status, const MetropolisTuning &tune,
                      hipStream_t stream);

int launch_log_u_table(float *approx, float *exact, hipStream_t stream);

int launch_prefix(int kind, const float *lw, int32_t *anc, int64_t P, uint64_t seed,
                  uint32_t instance, double *cumw, void *ws, int32_t *status,
                  hipStream_t stream);

int launch_log_sum_exp(const float *lw, int64_t P, double *out, void *ws, int32_t *status,
                       hipStream_t stream);

int launch_offspring(const int32_t *anc, int32_t *off, int64_t P, int32_t *status,
                     hipStream_t stream);

int launch_permute_copy(const int32_t *anc, const float *x_in, float *x_out, int64_t P, int32_t D,
                        int32_t *status, hipStream_t stream);

int launch_zero(void *ptr, size_t bytes, hipStream_t stream);

}  // namespace rs
