/*
 * resample.h -- C ABI of the MI355X (gfx950) particle-filter resampling library.
 *
 * Method: L. Murray, "GPU acceleration of the particle filter: the Metropolis
 * resampler", arXiv 1202.6163. The resampling step (Sec. 1, step 4) redraws P
 * particles with replacement using the weights as unnormalised probabilities.
 * The library represents the outcome by ancestors a_i (the parent of particle
 * i) or offspring counts o_j (Sec. 2), and copies the selected particles' state.
 *
 * Conventions (apply to every entry point unless stated otherwise)
 *  - Pointers marked [device] are device (HBM) pointers owned by the caller; the
 *    library never allocates, frees or retains them. Pointers marked [host] are
 *    host memory.
 *  - Indices are 0-based. Log-weights lw are binary32; -inf is a legal zero
 *    weight; lw is never modified.
 *  - Every call is asynchronous on `stream` (0 = the null stream) and returns
 *    before the kernels finish.
 *  - P = 0 is an empty resampling: RS_OK, nothing is launched or touched.
 *  - Argument errors are returned synchronously, before any launch:
 *      RS_EINVAL     null pointer, P < 0, P > 2^31 - 1, D < 1, overlapping
 *                    input and output buffers, unknown resampler kind;
 *      RS_EWORKSPACE workspace smaller than rs_workspace_bytes();
 *      RS_EHIP       a HIP launch failed (hipGetLastError after the launch).
 *  - Data errors are reported asynchronously: bits RS_FLAG_* are OR-ed into the
 *    caller's device status word (`status`, nullable). Outputs are then defined
 *    (every output element is written, no out-of-bounds access happens) but
 *    their values are unspecified.
 *  - Calls are re-entrant. Two calls that share a workspace must be ordered
 *    (same stream or explicit events).
 *  - Random numbers come from Philox4x32-10 (Salmon et al., SC'11) keyed by
 *    `seed`; `instance` separates independent resamplings under one seed. The
 *    result of a call is a pure function of its arguments.
 */
#ifndef PAPER_1202_6163_RESAMPLE_H
#define PAPER_1202_6163_RESAMPLE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t *hipStream_t;

/* return codes */
#define RS_OK 0
#define RS_EINVAL (-1)
#define RS_EWORKSPACE (-2)
#define RS_EHIP (-3)

/* device status bits */
#define RS_FLAG_NAN 1          /* a log-weight is NaN */
#define RS_FLAG_POSINF 2       /* a log-weight is +inf */
#define RS_FLAG_ALL_NEGINF 4   /* every log-weight is -inf (total weight zero) */
#define RS_FLAG_BAD_ANCESTOR 8 /* an ancestor index lies outside [0, P) */
#define RS_FLAG_INTERNAL 16    /* a library invariant failed (report as a bug) */

/* resampler kinds for rs_workspace_bytes() */
#define RS_STRATIFIED 0
#define RS_SYSTEMATIC 1
#define RS_MULTINOMIAL 2
#define RS_METROPOLIS 3
#define RS_LOG_SUM_EXP 4

/* Human-readable name of a return code. Never NULL. */
const char *rs_strerror(int code);

/* Library version as 10000 * major + 100 * minor + patch. */
int rs_version(void);

/*
 * Bytes of workspace the prefix-sum resamplers need for P particles: tile
 * partial sums, tile boundaries, per-tile draw counts, the fill table and,
 * for the multinomial resampler, the cumulative weights (pooled temporaries;
 * Sec. 3 replaces per-call allocations with reused pooled arrays). 0 for
 * RS_METROPOLIS. The workspace needs no initialisation: every call writes
 * what it reads, so one buffer serves any sequence of ordered calls.
 */
size_t rs_workspace_bytes(int64_t P, int resampler);

/* Zero-fill ws_bytes bytes of device memory on `stream` with a kernel (no
 * memset node, so it may be captured in a graph). Optional for workspaces. */
int rs_workspace_init(void *ws, size_t ws_bytes, hipStream_t stream);

/*
 * Metropolis resampler (Sec. 2, Fig. 1(d) and the paragraphs on B and its
 * convergence). Particle i runs its own chain from k = i for B iterations:
 * draw j uniformly over [0, P) and u uniformly on (0, 1); move to j iff
 * log u < lw[j] - lw[k]. Writes a_i = final k. No collective operation and one
 * kernel launch; B = 0 gives the identity.
 *   lw     [device] float[P]   log-weights
 *   anc    [device] int32[P]   ancestors (output)
 *   status [device] int32[1]   nullable; RS_FLAG_NAN / RS_FLAG_POSINF
 */
int resample_metropolis(const float *lw, int32_t *anc, int64_t P, uint32_t B, uint64_t seed,
                        uint32_t instance, int32_t *status, hipStream_t stream);

/*
 * Stratified resampler (Sec. 2, Fig. 1(b)): one uniform draw in each stratum
 * [i, i+1) * W / P of the cumulative weight, ancestor a_i = min{j : C_j > x_i}.
 * Ancestors come out sorted. Multi-kernel: a tile reduction, then a fused
 * scan and fill.
 *   lw     [device] float[P]    log-weights
 *   anc    [device] int32[P]    ancestors (output, non-decreasing)
 *   cumw   [device] double[P]   nullable; receives the cumulative weights
 *                               C_j = sum_{k<=j} exp(lw_k - max lw)
 *   ws     [device] workspace of ws_bytes >= rs_workspace_bytes(P, RS_STRATIFIED)
 *   status [device] int32[1]    nullable; RS_FLAG_NAN / POSINF / ALL_NEGINF
 */
int resample_stratified(const float *lw, int32_t *anc, int64_t P, uint64_t seed, uint32_t instance,
                        double *cumw, void *ws, size_t ws_bytes, int32_t *status,
                        hipStream_t stream);

/* Systematic resampler (Sec. 2, Fig. 1(c); Kitagawa): as stratified with one
 * shared offset for every stratum. Same arguments. */
int resample_systematic(const float *lw, int32_t *anc, int64_t P, uint64_t seed, uint32_t instance,
                        double *cumw, void *ws, size_t ws_bytes, int32_t *status,
                        hipStream_t stream);

/* Multinomial resampler (Sec. 2, Fig. 1(a)): P independent uniform draws on
 * [0, W), each located by binary search in the cumulative weights. Ancestors
 * are unsorted. Same arguments; cumw may be NULL (the workspace then holds C). */
int resample_multinomial(const float *lw, int32_t *anc, int64_t P, uint64_t seed,
                         uint32_t instance, double *cumw, void *ws, size_t ws_bytes,
                         int32_t *status, hipStream_t stream);

/*
 * Offspring counts from ancestors (Sec. 2: o_j = #{i : a_i = j}).
 *   anc    [device] int32[P], off [device] int32[P] (output), status nullable:
 *   RS_FLAG_BAD_ANCESTOR for entries outside [0, P), which are skipped.
 */
int ancestors_to_offspring(const int32_t *anc, int32_t *off, int64_t P, int32_t *status,
                           hipStream_t stream);

/*
 * Ancestor-indexed copy of particle state: x_out[i, :] = x_in[a_i, :], bit for
 * bit, rows of D binary32 values, row-major. x_in and x_out must not overlap.
 * Rows whose ancestor lies outside [0, P) are zero-filled and flagged
 * RS_FLAG_BAD_ANCESTOR.
 */
int permute_copy(const int32_t *anc, const float *x_in, float *x_out, int64_t P, int32_t D,
                 int32_t *status, hipStream_t stream);

/*
 * log sum_i exp(lw_i) in binary64 (the normalising constant of Sec. 1's
 * weighting step; a bootstrap filter adds it, minus log P, to its
 * log-likelihood each step). out [device] double[1].
 */
int rs_log_sum_exp(const float *lw, int64_t P, double *out, void *ws, size_t ws_bytes,
                   int32_t *status, hipStream_t stream); /* P >= 1 */

/*
 * Number of Metropolis iterations B (Sec. 2, eqs. (1)-(5)) for P particles
 * whose largest normalised weight is w_max, so that the chance a chain sits
 * at the heaviest particle is within eps of w_max from any start. Smallest
 * integer B >= 0 with lambda^B <= eps (alpha + beta) / max(alpha, beta),
 * alpha = (1 - w_max) / (P w_max), beta = 1 / P, lambda = 1 - alpha - beta.
 * Host function; returns 0 for invalid arguments.
 */
uint32_t metropolis_B(int64_t P, double w_max, double eps);

/*
 * Launch parameters of the Metropolis kernel (they change speed, never
 * results): threads per block (64..1024, multiple of 64), iterations each
 * lane prepares per round (2, 4, 8 or 16; one Philox block feeds two), the
 * largest P whose weights are staged in LDS (0 = never stage; P is also
 * capped by the device's LDS per block) and lanes cooperating on one chain
 * (1..64, power of two; 0 = chosen from P and B). The environment variables
 * RS_BLOCK, RS_UNROLL, RS_LDS_MAX_P and RS_LANES_PER_CHAIN override the
 * defaults at first use. Returns RS_EINVAL for values outside those ranges.
 */
typedef struct rs_metropolis_tuning {
    int32_t block;
    int32_t unroll;
    int64_t lds_max_p;
    int32_t lanes_per_chain;
} rs_metropolis_tuning;

int rs_metropolis_set_tuning(const rs_metropolis_tuning *t); /* t [host] */
int rs_metropolis_get_tuning(rs_metropolis_tuning *t);       /* t [host] */

/*
 * Self-check of the Metropolis acceptance test. The kernel decides
 * log u < d from the hardware log2 approximation whenever d is farther than
 * 2^-16 |log u| from it, and from the correctly rounded binary64-based log
 * otherwise; that is exact provided the approximation is within 2^-20
 * relative of the rounded log on every grid point. This writes both, for
 * all 2^23 grid points u = (2m + 1) 2^-24 in order of m, so a test can verify
 * the premise on the device it runs on.
 *   approx [device] float[2^23], nullable: hardware approximation of log u
 *   exact  [device] float[2^23], nullable: correctly rounded binary32 log u
 */
int rs_log_u_table(float *approx, float *exact, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* PAPER_1202_6163_RESAMPLE_H */
