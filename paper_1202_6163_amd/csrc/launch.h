// Internal launchers behind the C ABI (argument checking is done by the
// caller in capi.cpp; these only enqueue kernels). Return 0 or -3 (launch
// failure).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rs {

// 0 if no HIP error is pending, else -3 after recording the error for
// rs_last_hip_error().
int launch_status();
int record_hip_error(hipError_t e);

// Lets kernel `fn` launch with `bytes` of dynamic LDS on the current device
// (raises the kernel's limit once per device and size; thread-safe).
// Returns 0 or -3.
int allow_dynamic_lds(const void *fn, size_t bytes);

// Particle state rows to copy with the ancestors (x_out[i, :] = x_in[a_i, :]),
// D binary32 values per row; x_in == nullptr: no copy.
struct Rows {
    const float *x_in = nullptr;
    float *x_out = nullptr;
    int32_t D = 0;
};

struct MetropolisTuning {
    int32_t block;
    int32_t unroll;
    int64_t lds_max_p;
    int32_t lanes_per_chain;  // 0: chosen from P and B
};

int launch_metropolis(const float *lw, int32_t *anc, int64_t P, uint32_t B, uint64_t seed,
                      uint32_t instance, int32_t *status, const MetropolisTuning &tune,
                      hipStream_t stream, const Rows &rows = Rows());

int launch_log_u_table(float *approx, float *exact, hipStream_t stream);

// Metropolis with B read from device memory (B_dev, capped by B) after the
// launches before it on the stream computed it.
int launch_metropolis_dev_B(const float *lw, int32_t *anc, int64_t P, uint32_t B,
                            const uint32_t *B_dev, uint64_t seed, uint32_t instance,
                            int32_t *status, const MetropolisTuning &tune, hipStream_t stream,
                            const Rows &rows = Rows());

int launch_metropolis_adaptive(const float *lw, int32_t *anc, int64_t P, double eps,
                               uint32_t B_max, uint64_t seed, uint32_t instance, void *ws,
                               uint32_t *B_used, int32_t *status, const MetropolisTuning &tune,
                               hipStream_t stream);

// Which form the stratified/systematic single calls take: kPathAuto (the
// faster one: the launches), kPathLaunches (always the tile reduction, table
// and fill launches) or kPathOnePass (the clearing fill and the one
// resampling launch wherever it applies). wait_ns bounds a one-pass block's
// wait for the others' tile values before it reduces the missing tiles
// itself (< 0: the default). Process-wide; returns 0 or -1 (unknown path).
constexpr int kPathAuto = 0, kPathLaunches = 1, kPathOnePass = 2;
int set_prefix_path(int path, int64_t wait_ns);
int get_prefix_path();

int launch_prefix(int kind, const float *lw, int32_t *anc, int32_t *off, int64_t P, uint64_t seed,
                  uint32_t instance, double *cumw, void *ws, int32_t *status,
                  hipStream_t stream, const Rows &rows = Rows());

// Device address of this device's no-allocation workspace (the file-scope
// array in prefix.hip, RS_STATIC_SCRATCH_BYTES), looked up on first use.
// Returns 0, -1 (device index out of range) or -3.
int static_scratch(void **out);

int launch_log_sum_exp(const float *lw, int64_t P, double *out, void *ws, int32_t *status,
                       hipStream_t stream);
int launch_workspace_lse(const void *ws, int64_t P, double *out, hipStream_t stream);

// Sorted-weight variant: workspace sections (byte offsets) and the launcher
// (the radix sort's histograms live in the temp section). Returns 0 or -3.
struct SortedLayout {
    size_t prefix, keys_in, keys_out, idx_in, perm, a_sorted, temp, temp_bytes, total;
};
SortedLayout sorted_layout(int64_t P, int kind);
int launch_sorted(int kind, const float *lw, int32_t *anc, int64_t P, uint64_t seed,
                  uint32_t instance, void *ws, int32_t *status, hipStream_t stream);

// Tile reduction + table that leaves the eq. (5) iteration count (capped by
// B_max) in the workspace header (adaptive_B_slot) and in *B_used if given.
int launch_adaptive_B(const float *lw, int64_t P, double eps, uint32_t B_max, void *ws,
                      uint32_t *B_used, int32_t *status, hipStream_t stream);
const uint32_t *adaptive_B_slot(const void *ws);

int launch_offspring(const int32_t *anc, int32_t *off, int64_t P, int32_t *status,
                     hipStream_t stream);

// The same counts through a workspace without device-scope atomics
// (offspring.hip): its bytes (0 beyond 2^24 particles, where the launcher
// takes launch_offspring) and the four launches.
size_t offspring_workspace_bytes(int64_t P);
int launch_offspring_ws(const int32_t *anc, int32_t *off, int64_t P, void *ws, int32_t *status,
                        hipStream_t stream);

int launch_permute_copy(const int32_t *anc, const float *x_in, float *x_out, int64_t P, int32_t D,
                        int32_t *status, hipStream_t stream);

int launch_zero(void *ptr, size_t bytes, hipStream_t stream);

// Minimal-copy state update from offspring counts (inplace.hip): workspace
// bytes and the three launches.
size_t inplace_workspace_bytes(int64_t P);
int launch_offspring_update_inplace(const int32_t *off, float *x, int64_t P, int32_t D,
                                    int32_t *anc, void *ws, int32_t *status, hipStream_t stream);

int launch_gather_probe(const float *w, uint32_t n, uint32_t threads, uint32_t rounds,
                        uint32_t salt, float *out, hipStream_t stream);
int launch_philox_probe(uint64_t seed, uint32_t threads, uint32_t rounds, uint32_t *out,
                        hipStream_t stream);

// ---------------------------------------------------------------- batches
constexpr int kMetropolisKind = 3;  // RS_METROPOLIS
constexpr int kAdaptiveKind = 5;    // RS_METROPOLIS_ADAPTIVE (B from eq. (5) on the device)

// One instance of a batch as the kernels read it (device memory).
struct BatchInstance {
    const float *lw;
    int32_t *anc;
    int32_t *off;       // nullptr: no offspring
    const float *x_in;  // nullptr: no copy
    float *x_out;
    int32_t *status;
    char *ws;           // this instance's prefix workspace (stratified/systematic,
                        // and the table of an adaptive Metropolis instance)
    int64_t P;
    uint64_t seed;
    uint32_t B;         // iterations; the cap of eq. (5)'s count for kAdaptiveKind
    uint32_t instance;
    int32_t D;
    int32_t kind;
    double eps;         // eq. (5)'s tolerance (kAdaptiveKind)
};

struct BatchLaunch {
    const BatchInstance *insts;
    const int2 *tile_items;     // (instance, tile)
    const int32_t *table_items; // instance
    const int2 *main_items;     // (instance, fill block or Metropolis item)
    int32_t n_tile_items, n_table_items, n_main_items;
    int32_t blocks, unroll, chains_per_item;
    int64_t lds_max_p, max_table_tiles;
    size_t smem_main;
    uint32_t instance_add;  // added to every instance's Philox instance word
};

int launch_batch(const BatchLaunch &launch, hipStream_t stream);
int launch_batch_iterations(const BatchInstance *insts, int32_t n, uint32_t *out,
                            hipStream_t stream);
int launch_batch_log_mean_weight(const BatchInstance *insts, int32_t n, double *acc,
                                 hipStream_t stream);

// K filters of P particles each (K = 1: one filter); q_k: per-filter
// variances (device) or nullptr for the shared q.
int launch_filter_loglik(const double *lse, int32_t T, int64_t P, double *out, hipStream_t stream);
int launch_filter_init(float *x, int64_t P, int64_t K, int32_t D, uint64_t seed,
                       hipStream_t stream);

int launch_filter_step(const float *x_in, float *x_out, float *lw, int64_t P, int64_t K,
                       int32_t D, const double *A, const float *y, double q, const double *q_k,
                       double r, uint64_t seed, uint32_t t, hipStream_t stream);

}  // namespace rs
