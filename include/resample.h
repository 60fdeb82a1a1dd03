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
 *      RS_EINVAL     null pointer, P < 0, P > 2^31 - 1, D < 1, P * D above
 *                    2^40 state values (entry points that take rows), overlapping
 *                    input and output buffers, unknown resampler kind, a
 *                    workspace not 256-byte aligned (hipMalloc's blocks are);
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
#define RS_METROPOLIS_ADAPTIVE 5

/* Human-readable name of a return code. Never NULL. */
const char *rs_strerror(int code);

/* Library version as 10000 * major + 100 * minor + patch. */
int rs_version(void);

/* Description of the HIP error behind the calling thread's last RS_EHIP. */
const char *rs_last_hip_error(void);

/*
 * Bytes of workspace the prefix-sum resamplers need for P particles: tile
 * partial sums, tile boundaries, per-tile draw counts, the fill table and,
 * for the multinomial resampler, the cumulative weights with the search's
 * group ends, guide table and one part byte per draw (pooled temporaries;
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
 * Metropolis resampler with B chosen per call from the weights (Sec. 2:
 * eq. (5) for the largest normalised weight w_max and tolerance eps; the
 * paper warns that too small a B biases the sample). A tile reduction and a
 * one-block table compute W = sum_i exp(lw_i - max lw), so w_max = 1 / W,
 * and B = min(eq. (5), B_max) on the device; the chain kernel then reads B
 * from device memory (no host round trip; graph-capturable).
 *   eps    > 0; B_max caps the iteration count
 *   ws     [device] workspace of ws_bytes >= rs_workspace_bytes(P, RS_METROPOLIS_ADAPTIVE)
 *   B_used [device] uint32[1], nullable: the B that was used
 * Same results as resample_metropolis with that B.
 */
int resample_metropolis_adaptive(const float *lw, int32_t *anc, int64_t P, double eps,
                                 uint32_t B_max, uint64_t seed, uint32_t instance, void *ws,
                                 size_t ws_bytes, uint32_t *B_used, int32_t *status,
                                 hipStream_t stream);

/*
 * Stratified resampler (Sec. 2, Fig. 1(b)): one uniform draw in each stratum
 * [i, i+1) * W / P of the cumulative weight, ancestor a_i = min{j : C_j > x_i}.
 * Ancestors come out sorted. The paper gives this resampler's output as
 * offspring counts; it writes ancestors, offspring or both in the same pass.
 * Multi-kernel: a tile reduction, a table launch (more than 64 tiles),
 * then a fused scan and fill.
 *   lw     [device] float[P]    log-weights
 *   anc    [device] int32[P]    ancestors (output, non-decreasing), nullable
 *   off    [device] int32[P]    offspring o_j = #{i : a_i = j} (output), nullable;
 *                               anc and off must not both be NULL
 *   cumw   [device] double[P]   nullable; receives the cumulative weights
 *                               C_j = sum_{k<=j} exp(lw_k - max lw)
 *   ws     [device] workspace of ws_bytes >= rs_workspace_bytes(P, RS_STRATIFIED)
 *   status [device] int32[1]    nullable; RS_FLAG_NAN / POSINF / ALL_NEGINF
 *                               (then anc is the identity and every o_j is 1)
 */
int resample_stratified(const float *lw, int32_t *anc, int32_t *off, int64_t P, uint64_t seed,
                        uint32_t instance, double *cumw, void *ws, size_t ws_bytes,
                        int32_t *status, hipStream_t stream);

/* Systematic resampler (Sec. 2, Fig. 1(c); Kitagawa): as stratified with one
 * shared offset for every stratum. Same arguments. */
int resample_systematic(const float *lw, int32_t *anc, int32_t *off, int64_t P, uint64_t seed,
                        uint32_t instance, double *cumw, void *ws, size_t ws_bytes,
                        int32_t *status, hipStream_t stream);

/* Multinomial resampler (Sec. 2, Fig. 1(a)): P independent uniform draws on
 * [0, W), each located by binary search in the cumulative weights. Ancestors
 * are unsorted. Same arguments; cumw may be NULL (the workspace then holds C). */
int resample_multinomial(const float *lw, int32_t *anc, int64_t P, uint64_t seed,
                         uint32_t instance, double *cumw, void *ws, size_t ws_bytes,
                         int32_t *status, hipStream_t stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * stratified, systematic or multinomial resampler (kind RS_STRATIFIED,
 * RS_SYSTEMATIC or RS_MULTINOMIAL) exactly as resample_stratified /
 * resample_systematic / resample_multinomial compute it (the same kernels,
 * the same results), with no workspace argument: the workspace is a
 * library-owned device array of RS_STATIC_SCRATCH_BYTES per GPU, reserved
 * when the library is loaded on that GPU and held until the process ends.
 * The call allocates nothing (no hipMalloc or hipFree, here or in any
 * library routine it calls).
 *   lw, anc, off, cumw, status  as for resample_stratified (off: stratified
 *                               and systematic only)
 * Limits: rs_workspace_bytes(P, kind) <= RS_STATIC_SCRATCH_BYTES, which
 * holds for every kind up to P = 2^20 (and for stratified/systematic far
 * beyond); a larger P returns RS_EWORKSPACE before any launch.
 * Every call on one GPU shares that GPU's array (the last call's contents
 * stay; no call needs them cleared), so two calls that may overlap on one
 * GPU (different streams without ordering between them) race and give
 * unspecified results; order them like calls sharing a workspace.
 * Errors: RS_EINVAL, RS_EWORKSPACE, RS_EHIP (also if the array's address
 * cannot be found on the current device).
 */
#define RS_STATIC_SCRATCH_BYTES ((size_t)12 << 20)
int resample_prefix_static(int kind, const float *lw, int32_t *anc, int32_t *off, int64_t P,
                           uint64_t seed, uint32_t instance, double *cumw, int32_t *status,
                           hipStream_t stream);

/*
 * One resampling step with the state copy fused into the resampler's own
 * launches: the ancestors (and, for stratified/systematic, the offspring)
 * are exactly those of resample_metropolis / resample_stratified /
 * resample_systematic / resample_multinomial with the same arguments, and
 * x_out[i, :] = x_in[a_i, :] bit for bit, as permute_copy would write them
 * (Sec. 1: the selected particles are carried to the next time step). The
 * copy rides on the resampler's last kernel, where the ancestors are still
 * in registers or LDS, so they are not read back from HBM.
 *   kind   RS_METROPOLIS (B iterations), RS_STRATIFIED, RS_SYSTEMATIC or
 *          RS_MULTINOMIAL
 *   anc    [device] int32[P] ancestors (output, required)
 *   off    [device] int32[P] offspring (stratified/systematic only), nullable
 *   x_in   [device] float[P x D] row-major state, x_out the same shape (output);
 *          D >= 1; outputs overlap neither each other nor lw / x_in
 *   ws     [device] workspace of ws_bytes >= rs_workspace_bytes(P, kind);
 *          unused (may be NULL) for RS_METROPOLIS
 * Errors: RS_EINVAL, RS_EWORKSPACE, RS_EHIP. Graph-capturable.
 */
int resample_and_copy(int kind, const float *lw, int32_t *anc, int32_t *off, int64_t P, uint32_t B,
                      uint64_t seed, uint32_t instance, const float *x_in, float *x_out,
                      int32_t D, void *ws, size_t ws_bytes, int32_t *status, hipStream_t stream);

/*
 * Sorted-weight variant of a prefix-sum resampler (Sec. 3 compares the
 * resamplers with the weights sorted before the prefix sum, which speeds up
 * the multinomial bisection, and without). The particles are ordered by
 * decreasing log-weight, equal weights by index (-0 counts as +0); the
 * resampler `kind` (RS_STRATIFIED, RS_SYSTEMATIC or RS_MULTINOMIAL) runs on
 * the weights in that order with the given seed and instance; anc receives
 * the chosen particles' original indices. The sort is the library's own
 * stable radix sort (four 8-bit passes of histogram, scan and scatter
 * launches); the call allocates nothing and issues no memory fills, so it
 * can be captured in a graph.
 *   lw, anc  [device] float[P] / int32[P], not overlapping
 *   ws       [device] workspace of ws_bytes >= rs_sorted_workspace_bytes(P, kind)
 *   status   [device] int32[1], nullable; flagged inputs give identity ancestors
 * Errors: RS_EINVAL, RS_EWORKSPACE, RS_EHIP.
 */
size_t rs_sorted_workspace_bytes(int64_t P, int kind);
int resample_sorted(int kind, const float *lw, int32_t *anc, int64_t P, uint64_t seed,
                    uint32_t instance, void *ws, size_t ws_bytes, int32_t *status,
                    hipStream_t stream);

/*
 * Offspring counts from ancestors (Sec. 2: o_j = #{i : a_i = j}).
 *   anc    [device] int32[P], off [device] int32[P] (output), status nullable:
 *   RS_FLAG_BAD_ANCESTOR for entries outside [0, P), which are skipped.
 */
int ancestors_to_offspring(const int32_t *anc, int32_t *off, int64_t P, int32_t *status,
                           hipStream_t stream);

/*
 * The same offspring counts (bit for bit, flags included) through a
 * workspace: the ancestors are grouped by buckets of particles, then each
 * bucket's counts are formed on chip and written whole, so random ancestors
 * cost no device-scope atomics and off needs no clearing. Four launches;
 * graph-capturable. Beyond P = 2^24, rs_offspring_workspace_bytes is 0 and the
 * call runs as ancestors_to_offspring (ws may then be NULL).
 *   ws     [device] workspace of ws_bytes >= rs_offspring_workspace_bytes(P),
 *          256-byte aligned; must not overlap anc or off
 * Errors: RS_EINVAL, RS_EWORKSPACE, RS_EHIP.
 */
size_t rs_offspring_workspace_bytes(int64_t P);
int ancestors_to_offspring_ws(const int32_t *anc, int32_t *off, int64_t P, void *ws,
                              size_t ws_bytes, int32_t *status, hipStream_t stream);

/*
 * Ancestor-indexed copy of particle state: x_out[i, :] = x_in[a_i, :], bit for
 * bit, rows of D binary32 values, row-major. x_in and x_out must not overlap.
 * Rows whose ancestor lies outside [0, P) are zero-filled and flagged
 * RS_FLAG_BAD_ANCESTOR.
 */
int permute_copy(const int32_t *anc, const float *x_in, float *x_out, int64_t P, int32_t D,
                 int32_t *status, hipStream_t stream);

/*
 * Minimal-copy state update from offspring counts (Sec. 2 gives a
 * resampler's output as offspring o_j, the number of copies of particle j,
 * and notes that offspring and ancestors convert into each other). After
 * resampling every particle carries weight 1 / P, so the new population is
 * the multiset {x_j repeated o_j times} and slot order is free. This update
 * rewrites x IN PLACE into that multiset moving only the rows that must
 * change: row j stays in slot j whenever o_j >= 1, and each slot i with
 * o_i = 0 (a hole) receives one extra copy (o_j - 1 of them for each j with
 * o_j >= 2), the holes in increasing slot order paired with the extras in
 * increasing order of j. HBM traffic is about 8D bytes per hole (plus 12 to
 * 16 bytes per particle of counts and indices) instead of 4 + 8D per particle
 * for permute_copy into a second buffer.
 *   off    [device] int32[P]   offspring counts (as the stratified/systematic
 *                              resamplers or ancestors_to_offspring write them)
 *   x      [device] float[P x D] row-major state, updated in place; D >= 1
 *   anc    [device] int32[P]   nullable; receives the particle whose row slot i
 *                              holds afterwards (i itself where o_i >= 1)
 *   ws     [device] workspace of ws_bytes >= rs_inplace_workspace_bytes(P)
 *   status [device] int32[1]   nullable; RS_FLAG_BAD_ANCESTOR if a count is
 *                              negative or the counts do not sum to P (then x
 *                              is unchanged and anc is the identity)
 * off, x, anc and ws must not overlap. Three launches; graph-capturable.
 */
size_t rs_inplace_workspace_bytes(int64_t P);
int offspring_update_inplace(const int32_t *off, float *x, int64_t P, int32_t D, int32_t *anc,
                             void *ws, size_t ws_bytes, int32_t *status, hipStream_t stream);

/*
 * log sum_i exp(lw_i) in binary64 (the normalising constant of Sec. 1's
 * weighting step; a bootstrap filter adds it, minus log P, to its
 * log-likelihood each step). out [device] double[1].
 */
int rs_log_sum_exp(const float *lw, int64_t P, double *out, void *ws, size_t ws_bytes,
                   int32_t *status, hipStream_t stream);
/*
 * The log sum_i exp(lw_i) that the last call on workspace ws computed, for
 * P particles, in binary64 (the same bits rs_log_sum_exp gives): every
 * prefix resampler (stratified, systematic, multinomial, also through
 * resample_and_copy and resample_batch) and resample_metropolis_adaptive
 * reduce the weights anyway, so a filter reads its likelihood factor here
 * instead of reducing them twice. NaN (NaN or +inf weights) or -inf (all
 * -inf) when that call flagged its input.
 *   ws  [device] the workspace of that call, P its particle count
 *   out [device] double[1]. Stream-ordered after that call; graph-capturable.
 */
int rs_workspace_log_sum_exp(const void *ws, int64_t P, double *out, hipStream_t stream); /* P >= 1 */

/*
 * Batched resampling: many independent instances of uneven size in one graph
 * replay of three persistent launches (tile reductions, per-instance tables,
 * then Metropolis chains and stratified/systematic fills with the state copy
 * fused in). Particle MCMC runs many filters, each resampling at every step
 * (Sec. 1); batching removes the per-instance launch overhead the paper
 * observes for small resamplings (Sec. 3). Every instance's ancestors and
 * copied rows are bit-identical to the corresponding single call
 * (resample_metropolis / resample_stratified / resample_systematic, then
 * permute_copy) with the same seed and instance; an RS_METROPOLIS_ADAPTIVE
 * instance equals resample_metropolis_adaptive (B from eq. (5) for its own
 * weights, capped by its B) followed by permute_copy.
 *
 * Usage: fill rs_instance[n] on the host; size the device plan and workspace
 * with rs_batch_plan_bytes / rs_batch_workspace_bytes; rs_batch_plan_init
 * validates the instances, builds the work lists and uploads them; then
 * resample_batch (any number of times, capturable in a graph) runs them.
 */
typedef struct rs_instance {
    const float *lw;    /* [device] float[P] log-weights */
    int32_t *anc;       /* [device] int32[P] ancestors (output) */
    int32_t *off;       /* [device] int32[P] offspring (output; stratified and
                           systematic only), or NULL */
    const float *x_in;  /* [device] float[P x D] state, or NULL: no copy */
    float *x_out;       /* [device] float[P x D] copied state (output) */
    int32_t *status;    /* [device] int32[1] flags of this instance, nullable */
    int64_t P;          /* 0 <= P <= 2^31 - 1 */
    int32_t D;          /* state width when x_in != NULL (>= 1) */
    int32_t kind;       /* RS_METROPOLIS, RS_METROPOLIS_ADAPTIVE, RS_STRATIFIED or
                           RS_SYSTEMATIC */
    uint32_t B;         /* Metropolis iterations; for RS_METROPOLIS_ADAPTIVE the cap
                           B_max of eq. (5)'s count (as resample_metropolis_adaptive) */
    uint32_t instance;  /* Philox instance word */
    uint64_t seed;      /* Philox key */
    double eps;         /* RS_METROPOLIS_ADAPTIVE: eq. (5)'s tolerance (> 0); else unused */
} rs_instance;

typedef struct rs_batch_tuning {
    int32_t chains_per_item; /* Metropolis chains per work item: 256, 512, 1024 or 2048 */
    int32_t unroll;          /* Metropolis iterations per round: 2, 4, 8 or 16 */
    int64_t lds_max_p;       /* stage an instance's weights in LDS when P <= this (<= 32768) */
    int32_t blocks;          /* persistent blocks per launch; 0 = 8 per compute unit */
} rs_batch_tuning;

/* Filled by rs_batch_plan_init; plain data (device pointers and counts). */
typedef struct rs_batch_plan {
    const void *dev;           /* device plan buffer */
    int32_t n_instances;
    int32_t n_tile_items;
    int32_t n_table_items;
    int32_t n_main_items;
    int32_t blocks;
    int32_t unroll;
    int32_t chains_per_item;
    int32_t reserved;
    int64_t lds_max_p;
    int64_t max_table_tiles;
    uint64_t off_tile_items;   /* byte offsets inside dev */
    uint64_t off_table_items;
    uint64_t off_main_items;
    uint64_t smem_main;
} rs_batch_plan;

/* Device bytes of the plan buffer (descriptors + work lists); 0 if invalid.
 * t may be NULL for the defaults. */
size_t rs_batch_plan_bytes(const rs_instance *descs, int32_t n, const rs_batch_tuning *t);
/* Device bytes of workspace for the batch's stratified/systematic instances. */
size_t rs_batch_workspace_bytes(const rs_instance *descs, int32_t n);
/*
 * Validate descs[n] (host array), build the work lists and copy them to
 * plan_dev (device, plan_bytes >= rs_batch_plan_bytes). ws (device,
 * ws_bytes >= rs_batch_workspace_bytes) is carved into per-instance
 * workspaces. With host_staging == NULL the upload is synchronous on
 * `stream`; otherwise host_staging (pinned host memory of plan_bytes bytes)
 * receives the plan and is copied asynchronously on `stream`, and must stay
 * untouched until that copy completes. Errors: RS_EINVAL (bad instance or
 * tuning), RS_EWORKSPACE (plan_bytes or ws_bytes too small), RS_EHIP.
 */
int rs_batch_plan_init(rs_batch_plan *plan, const rs_instance *descs, int32_t n,
                       const rs_batch_tuning *t, void *plan_dev, size_t plan_bytes, void *ws,
                       size_t ws_bytes, void *host_staging, hipStream_t stream);
/* Run a batch (asynchronous on `stream`; graph-capturable). */
int resample_batch(const rs_batch_plan *plan, hipStream_t stream);
/* As resample_batch with instance_add added to every instance's Philox
 * instance word (the same plan serves every time step of a set of filters:
 * instance = t gives each step fresh draws). resample_batch is
 * resample_batch_at(plan, 0, stream). */
int resample_batch_at(const rs_batch_plan *plan, uint32_t instance_add, hipStream_t stream);
/*
 * acc[k] += lse_k - log P_k for every instance k of the plan's last run: the
 * log of its mean weight, the likelihood factor of Sec. 1's weighting step
 * (lse_k = log sum_i exp(lw_i) from the instance's table). Stratified and
 * systematic instances only; Metropolis and empty instances add NaN, and
 * flagged weights NaN (NaN or +inf present) or -inf (all -inf).
 *   acc [device] double[n_instances]. Graph-capturable.
 */
int rs_batch_log_mean_weight(const rs_batch_plan *plan, double *acc, hipStream_t stream);
/*
 * out[k] = the Metropolis iterations instance k ran in the plan's last run
 * (Sec. 2: the B of eq. (5) an RS_METROPOLIS_ADAPTIVE instance computed from
 * its weights, capped by its B; the fixed B of an RS_METROPOLIS instance; 0
 * for the prefix resamplers and empty instances).
 *   out [device] uint32[n_instances]. Stream-ordered after that run.
 */
int rs_batch_iterations(const rs_batch_plan *plan, uint32_t *out, hipStream_t stream);

/*
 * Bootstrap particle filter around the resampler (Sec. 1: initialisation,
 * propagation, weighting) for the linear-Gaussian model
 *   x_0 ~ N(0, I),  x_t = A x_{t-1} + N(0, q I),  y_t = x_t + N(0, r I),
 * with the transition as proposal, so lw_i = log N(y_t; x_t^i, r I).
 * Gaussian draws: Box-Muller on Philox block (i, t, h, 5) for components
 * 4h..4h+3, u1 = (r + 1/2) 2^-32, u2 = r' 2^-32 (t = 0: initial state).
 *   x, x_in, x_out [device] float[P x D] row-major, 1 <= D <= 64; x_in and
 *                  x_out must not overlap
 *   lw             [device] float[P] log-weights (output)
 *   A              [device] double[D x D] row-major transition matrix
 *   y              [device] float[D] observation at time t
 *   q, r           noise variances (q >= 0, r > 0); t >= 1 for a step
 */
int filter_init(float *x, int64_t P, int32_t D, uint64_t seed, hipStream_t stream);
/*
 * K filters at once (particle MCMC evaluates K parameter values per step):
 * filter k holds rows [k P, (k+1) P) of x (and of lw), draws with Philox key
 * seed + k and uses the noise variance q[k] (q: device double[K], each >= 0),
 * so it computes exactly what filter_init / filter_propagate_weight compute
 * for one filter with key seed + k and q = q[k]. A, y, r are shared.
 */
int filter_init_batch(float *x, int32_t K, int64_t P, int32_t D, uint64_t seed,
                      hipStream_t stream);
int filter_propagate_weight_batch(const float *x_in, float *x_out, float *lw, int32_t K, int64_t P,
                                  int32_t D, const double *A, const float *y, const double *q,
                                  double r, uint64_t seed, uint32_t t, hipStream_t stream);
int filter_propagate_weight(const float *x_in, float *x_out, float *lw, int64_t P, int32_t D,
                            const double *A, const float *y, double q, double r, uint64_t seed,
                            uint32_t t, hipStream_t stream);
/*
 * The filter's log-likelihood estimate (Sec. 1: the weights' sum at each
 * step, the normalising constant of the weighting step, estimates the
 * observation density): out = sum_t (lse_t - log P), added in time order,
 * where lse_t = log sum_i exp(lw_i) of step t (rs_workspace_log_sum_exp or
 * rs_log_sum_exp). A NaN or -inf factor propagates.
 *   lse [device] double[T], T >= 0; out [device] double[1] (output); P >= 1
 * Errors: RS_EINVAL (null pointers, T < 0, P out of range, out inside lse).
 */
int filter_loglik(const double *lse, int32_t T, int64_t P, double *out, hipStream_t stream);

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
 * Form of the stratified and systematic single calls (resample_stratified,
 * resample_systematic, resample_and_copy, resample_prefix_static; the
 * results are the same bits in every form). Sec. 2 notes that the prefix sum
 * needs thread communication and several kernel launches, and Sec. 3 that
 * launch overhead dominated at small sizes; up to P = 2^20 these calls can
 * run as ONE resampling launch in which the blocks exchange their tile sums
 * through device memory (tagged words, no fence) instead of through kernel
 * boundaries, after a small fill kernel that clears those words.
 *   path    RS_PATH_AUTO (the faster form as measured on the MI355X: the
 *           launches at every size so far), RS_PATH_LAUNCHES (always the tile
 *           reduction, table and fill launches) or RS_PATH_ONEPASS (the one
 *           launch wherever it applies: P <= 2^20 and the device holds all
 *           its blocks at once; else the launches)
 *   wait_ns bound on a one-pass block's wait for the other blocks' tile sums
 *           before it computes the missing ones itself (< 0: the default,
 *           100 us; 0: never wait). It changes speed, never results.
 * Process-wide. Returns RS_OK or RS_EINVAL (unknown path).
 */
#define RS_PATH_AUTO 0
#define RS_PATH_LAUNCHES 1
#define RS_PATH_ONEPASS 2
int rs_prefix_set_path(int path, int64_t wait_ns);
int rs_prefix_get_path(void); /* the current path */

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

/*
 * Measurement probes for the Metropolis roofline (not resamplers). The
 * gather probe performs threads x rounds x 8 random 4-byte loads from
 * w[0..n) (xorshift indices through the same index map as the proposals);
 * the Philox probe computes threads x rounds x 4 Philox4x32-10 blocks. Each
 * thread writes one folded word to out[threads] [device]. threads is a
 * multiple of 256. Timing them gives the device's random-gather and Philox
 * rates, the two ceilings of a Metropolis iteration.
 */
int rs_probe_gather(const float *w, int64_t n, int64_t threads, int64_t rounds, uint32_t salt,
                    float *out, hipStream_t stream);
int rs_probe_philox(uint64_t seed, int64_t threads, int64_t rounds, uint32_t *out,
                    hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* PAPER_1202_6163_RESAMPLE_H */
