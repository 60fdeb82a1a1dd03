/*
 * resample_oracle.c -- CPU oracle for the particle-filter resampling stage of
 * L. Murray, "GPU acceleration of the particle filter: the Metropolis
 * resampler" (arXiv 1202.6163).
 *
 * TEST INFRASTRUCTURE. This file is a plain, slow, single-threaded statement of
 * what the resampling path computes. Only the test suite, the smoke check and
 * the benchmark's CPU-baseline leg may load it; the HIP library never includes,
 * links or calls it, and it shares no source with the HIP library.
 *
 * The same source is also built a second time with OpenMP (liboracle_omp.so)
 * for the all-core CPU baseline: only the particle loops of the Metropolis
 * resampler and of the state copy carry a pragma, each iteration is
 * independent (counter-based random numbers, disjoint output rows), so that
 * build returns the same bits; the single-threaded build ignores the pragmas.
 *
 * Arithmetic rules: IEEE-754 binary32 / binary64 with round-to-nearest-even,
 * built with -O2 -ffp-contract=off -fno-fast-math on SSE2 (no x87 excess
 * precision), so every expression below rounds exactly where it is written.
 *
 * Where the paper is silent (its pseudocode listing is not reproduced in the
 * text), the readings used here are:
 *   - random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) keyed by
 *     the 64-bit seed, counter (c0, c1, c2, c3) = (particle index or index group,
 *     instance, draw block, tag); the paper used a stateful Tausworthe stream.
 *   - Metropolis: chain k starts at its own index, proposes j uniformly over all
 *     P indices (Sec. 2, the transition-matrix derivation assumes this), accepts
 *     iff log u < lw[j] - lw[k] in binary32 with log u correctly rounded.
 *   - inverse-CDF search: a(x) = min{j : C_j > x}; if x >= C_{P-1}, the first j
 *     with C_j = C_{P-1} (never a zero-weight particle).
 *   - stratified, systematic, multinomial draws as documented per function.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_FLAG_NAN 1
#define ORACLE_FLAG_POSINF 2
#define ORACLE_FLAG_ALL_NEGINF 4
#define ORACLE_FLAG_BAD_ANCESTOR 8

#define ORACLE_EINVAL (-1)

/* Counter tags: which part of the method a Philox block feeds. */
#define TAG_METROPOLIS 1u
#define TAG_STRATIFIED 2u
#define TAG_SYSTEMATIC 3u
#define TAG_MULTINOMIAL 4u
#define TAG_FILTER_NOISE 5u

/* ------------------------------------------------------------------------ */
/* Philox4x32-10, as defined by Salmon et al. (SC'11): ten rounds of two     */
/* 32x32->64 multiplications with the round key bumped by the Weyl constants */
/* between rounds.                                                           */
/* ------------------------------------------------------------------------ */

void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    const uint32_t mult0 = 0xD2511F53u, mult1 = 0xCD9E8D57u;
    const uint32_t weyl0 = 0x9E3779B9u, weyl1 = 0xBB67AE85u;
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += weyl0;
            k1 += weyl1;
        }
        uint64_t prod0 = (uint64_t)mult0 * (uint64_t)c0;
        uint64_t prod1 = (uint64_t)mult1 * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(prod0 >> 32), lo0 = (uint32_t)prod0;
        uint32_t hi1 = (uint32_t)(prod1 >> 32), lo1 = (uint32_t)prod1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* One Philox block for (seed, counter). */
static void draw_block(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t tag,
                       uint32_t out[4])
{
    uint32_t ctr[4] = {c0, c1, c2, tag};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    oracle_philox4x32_10(ctr, key, out);
}

/* ------------------------------------------------------------------------ */
/* Draw conversions                                                          */
/* ------------------------------------------------------------------------ */

/* Uniform index in [0, P) from a 32-bit word: the high word of r * P. */
uint32_t oracle_index(uint32_t r, int64_t P)
{
    return (uint32_t)(((uint64_t)r * (uint64_t)P) >> 32);
}

/* Uniform u on the open grid {(2m+1) 2^-24 : 0 <= m < 2^23}, exact in binary32. */
float oracle_metropolis_u(uint32_t r)
{
    uint32_t m = r >> 9;
    return (float)(2u * m + 1u) * 0x1p-24f;
}

/* Correctly rounded binary32 natural logarithm of u, via binary64. */
float oracle_log_u(float u)
{
    return (float)log((double)u);
}

/* Fill the whole u grid with L(u), in grid order (m = 0 .. 2^23-1). */
void oracle_log_u_table(float *out)
{
    for (uint32_t m = 0; m < (1u << 23); ++m) {
        float u = (float)(2u * m + 1u) * 0x1p-24f;
        out[m] = oracle_log_u(u);
    }
}

/* Count, for each j in [0, P), how many of the 2^32 words map to index j. */
void oracle_index_histogram(int64_t P, uint64_t *counts)
{
    memset(counts, 0, (size_t)P * sizeof(uint64_t));
    uint32_t r = 0;
    do {
        counts[oracle_index(r, P)] += 1;
        r += 1;
    } while (r != 0);
}

/* ------------------------------------------------------------------------ */
/* Input screening shared by every resampler (status flags).                 */
/* ------------------------------------------------------------------------ */

static int32_t screen_weights(const float *lw, int64_t P)
{
    int32_t flags = 0;
    int any_above_neginf = 0;
    for (int64_t i = 0; i < P; ++i) {
        float v = lw[i];
        if (isnan(v)) flags |= ORACLE_FLAG_NAN;
        else if (isinf(v) && v > 0) flags |= ORACLE_FLAG_POSINF;
        if (!(isinf(v) && v < 0)) any_above_neginf = 1;
    }
    if (!any_above_neginf) flags |= ORACLE_FLAG_ALL_NEGINF;
    return flags;
}

/* ------------------------------------------------------------------------ */
/* Metropolis resampler (Sec. 2: Fig. 1(d); the paragraph on B; the          */
/* convergence analysis assumes a uniform proposal over all P indices and    */
/* acceptance by the weight ratio).                                          */
/*                                                                           */
/* Chain i starts at k = i. Iteration n uses Philox block n/2 at counter     */
/* (i, instance, n/2, 1): words (r0, r1) for even n, (r2, r3) for odd n; the */
/* first word gives the proposal j, the second the uniform u. The move is    */
/* accepted iff L(u) < lw[j] - lw[k], the difference rounded to binary32.    */
/* ------------------------------------------------------------------------ */

static int32_t metropolis_chain(const float *lw, int64_t P, uint32_t B, uint64_t seed,
                                uint32_t instance, int64_t i)
{
    int64_t k = i;
    float lk = lw[i];
    uint32_t r[4] = {0, 0, 0, 0};
    for (uint32_t n = 0; n < B; ++n) {
        if ((n & 1u) == 0) draw_block(seed, (uint32_t)i, instance, n >> 1, TAG_METROPOLIS, r);
        uint32_t rj = (n & 1u) ? r[2] : r[0];
        uint32_t ru = (n & 1u) ? r[3] : r[1];
        int64_t j = oracle_index(rj, P);
        float d = lw[j] - lk;
        float logu = oracle_log_u(oracle_metropolis_u(ru));
        if (logu < d) {
            k = j;
            lk = lw[j];
        }
    }
    return (int32_t)k;
}

int oracle_metropolis(const float *lw, int32_t *anc, int64_t P, uint32_t B, uint64_t seed,
                      uint32_t instance, int32_t *status)
{
    if (!lw || !anc || P < 1 || P > INT32_MAX) return ORACLE_EINVAL;
    int32_t flags = screen_weights(lw, P) & (ORACLE_FLAG_NAN | ORACLE_FLAG_POSINF);
    /* chains are independent: the OpenMP build (CPU baseline only) splits them */
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < P; ++i) anc[i] = metropolis_chain(lw, P, B, seed, instance, i);
    if (status) *status |= flags;
    return 0;
}

/* The chains of the particles listed in idx[0..n) only (same results as   */
/* the full resampling at those positions).                                */
int oracle_metropolis_subset(const float *lw, int64_t P, uint32_t B, uint64_t seed,
                             uint32_t instance, const int64_t *idx, int64_t n, int32_t *out)
{
    if (!lw || !idx || !out || P < 1 || P > INT32_MAX || n < 0) return ORACLE_EINVAL;
    for (int64_t s = 0; s < n; ++s) {
        if (idx[s] < 0 || idx[s] >= P) return ORACLE_EINVAL;
        out[s] = metropolis_chain(lw, P, B, seed, instance, idx[s]);
    }
    return 0;
}

/* Many independent resamplings of one weight vector, instances inst0 ..   */
/* inst0 + n_inst - 1, written row by row into anc[n_inst * P].            */
int oracle_metropolis_many(const float *lw, int32_t *anc, int64_t P, uint32_t B, uint64_t seed,
                           uint32_t inst0, int64_t n_inst)
{
    if (!lw || !anc || P < 1 || P > INT32_MAX || n_inst < 0) return ORACLE_EINVAL;
    for (int64_t s = 0; s < n_inst; ++s)
        for (int64_t i = 0; i < P; ++i)
            anc[s * P + i] = metropolis_chain(lw, P, B, seed, inst0 + (uint32_t)s, i);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Normalising constant and cumulative weights (Sec. 1, the resampling step  */
/* uses the weights as unnormalised probabilities; Sec. 2, the collective    */
/* prefix sum the multinomial, stratified and systematic resamplers need).   */
/*                                                                           */
/* m = max lw; w_j = exp(lw_j - m) in binary64 (the difference is exact);    */
/* C_j = w_0 + ... + w_j summed left to right in binary64.                   */
/* ------------------------------------------------------------------------ */

int oracle_cumulative(const float *lw, int64_t P, double *C, float *m_out, int32_t *status)
{
    if (!lw || !C || P < 1) return ORACLE_EINVAL;
    int32_t flags = screen_weights(lw, P);
    if (status) *status |= flags;
    if (flags) return flags;
    float m = -INFINITY;
    for (int64_t i = 0; i < P; ++i)
        if (lw[i] > m) m = lw[i];
    double acc = 0.0;
    for (int64_t j = 0; j < P; ++j) {
        acc += exp((double)lw[j] - (double)m);
        C[j] = acc;
    }
    if (m_out) *m_out = m;
    return 0;
}

/* The same sum in 80-bit extended precision, to bound the oracle's own      */
/* rounding error.                                                           */
int oracle_cumulative_extended(const float *lw, int64_t P, double *C_hi, double *C_lo)
{
    if (!lw || !C_hi || P < 1) return ORACLE_EINVAL;
    if (screen_weights(lw, P)) return ORACLE_EINVAL;
    float m = -INFINITY;
    for (int64_t i = 0; i < P; ++i)
        if (lw[i] > m) m = lw[i];
    long double acc = 0.0L;
    for (int64_t j = 0; j < P; ++j) {
        acc += expl((long double)lw[j] - (long double)m);
        C_hi[j] = (double)acc;
        if (C_lo) C_lo[j] = (double)(acc - (long double)C_hi[j]);
    }
    return 0;
}

/* Inverse-CDF search rule: a(x) = min{j : C_j > x} when x < C_{P-1};        */
/* otherwise the first j with C_j = C_{P-1}. C is non-decreasing, so the     */
/* minimum is found by bisection.                                            */
int64_t oracle_search(const double *C, int64_t P, double x)
{
    double total = C[P - 1];
    int64_t lo = 0, hi = P - 1;
    if (x < total) {
        while (lo < hi) { /* first index with C > x */
            int64_t mid = lo + (hi - lo) / 2;
            if (C[mid] > x) hi = mid;
            else lo = mid + 1;
        }
    } else {
        while (lo < hi) { /* first index with C == total */
            int64_t mid = lo + (hi - lo) / 2;
            if (C[mid] >= total) hi = mid;
            else lo = mid + 1;
        }
    }
    return lo;
}

/* ------------------------------------------------------------------------ */
/* Draw points x_i for the three prefix-sum resamplers (Sec. 2, Fig. 1(a-c)). */
/*   stratified:  x_i = (i + U_i) * (W / P), U_i from word i mod 4 of block   */
/*                (i / 4, instance, 0, 2), U = r * 2^-32.                     */
/*   systematic:  x_i = (i + U) * (W / P), one U from word 0 of block         */
/*                (0, instance, 0, 3).                                        */
/*   multinomial: x_i = U_i * W, U_i a 53-bit uniform from words (0,1) (even  */
/*                i) or (2,3) (odd i) of block (i / 2, instance, 0, 4).       */
/* kind: 0 stratified, 1 systematic, 2 multinomial.                          */
/* ------------------------------------------------------------------------ */

int oracle_draw_points(int kind, int64_t P, double W, uint64_t seed, uint32_t instance, double *x)
{
    if (!x || P < 1 || kind < 0 || kind > 2) return ORACLE_EINVAL;
    uint32_t r[4];
    if (kind == 0) {
        double delta = W / (double)P;
        for (int64_t i = 0; i < P; ++i) {
            draw_block(seed, (uint32_t)(i >> 2), instance, 0, TAG_STRATIFIED, r);
            double U = (double)r[i & 3] * 0x1p-32;
            x[i] = ((double)i + U) * delta;
        }
    } else if (kind == 1) {
        double delta = W / (double)P;
        draw_block(seed, 0, instance, 0, TAG_SYSTEMATIC, r);
        double U = (double)r[0] * 0x1p-32;
        for (int64_t i = 0; i < P; ++i) x[i] = ((double)i + U) * delta;
    } else {
        for (int64_t i = 0; i < P; ++i) {
            draw_block(seed, (uint32_t)(i >> 1), instance, 0, TAG_MULTINOMIAL, r);
            uint32_t ra = (i & 1) ? r[2] : r[0];
            uint32_t rb = (i & 1) ? r[3] : r[1];
            double U = (double)(((uint64_t)ra << 21) | (uint64_t)(rb >> 11)) * 0x1p-53;
            x[i] = U * W;
        }
    }
    return 0;
}

static int prefix_resampler(int kind, const float *lw, int32_t *anc, int64_t P, uint64_t seed,
                            uint32_t instance, double *cumw, int32_t *status)
{
    if (!lw || !anc || P < 1 || P > INT32_MAX) return ORACLE_EINVAL;
    double *C = cumw ? cumw : (double *)malloc((size_t)P * sizeof(double));
    double *x = (double *)malloc((size_t)P * sizeof(double));
    if (!C || !x) {
        if (!cumw) free(C);
        free(x);
        return ORACLE_EINVAL;
    }
    int32_t flags = 0;
    int rc = oracle_cumulative(lw, P, C, NULL, &flags);
    if (status) *status |= flags;
    if (rc == 0) {
        oracle_draw_points(kind, P, C[P - 1], seed, instance, x);
        for (int64_t i = 0; i < P; ++i) anc[i] = (int32_t)oracle_search(C, P, x[i]);
    } else {
        for (int64_t i = 0; i < P; ++i) anc[i] = (int32_t)i;
    }
    if (!cumw) free(C);
    free(x);
    return rc > 0 ? 0 : rc;
}

int oracle_stratified(const float *lw, int32_t *anc, int64_t P, uint64_t seed, uint32_t instance,
                      double *cumw, int32_t *status)
{
    return prefix_resampler(0, lw, anc, P, seed, instance, cumw, status);
}

int oracle_systematic(const float *lw, int32_t *anc, int64_t P, uint64_t seed, uint32_t instance,
                      double *cumw, int32_t *status)
{
    return prefix_resampler(1, lw, anc, P, seed, instance, cumw, status);
}

int oracle_multinomial(const float *lw, int32_t *anc, int64_t P, uint64_t seed, uint32_t instance,
                       double *cumw, int32_t *status)
{
    return prefix_resampler(2, lw, anc, P, seed, instance, cumw, status);
}

/* ------------------------------------------------------------------------ */
/* Offspring counts and ancestor-indexed copy (Sec. 2: o_i is the number of  */
/* offspring of particle i, a_i the ancestor of particle i; the selected     */
/* ancestors' states are what propagate to the next time).                   */
/* ------------------------------------------------------------------------ */

int oracle_ancestors_to_offspring(const int32_t *anc, int32_t *off, int64_t P)
{
    if (!anc || !off || P < 1) return ORACLE_EINVAL;
    for (int64_t j = 0; j < P; ++j) off[j] = 0;
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
    for (int64_t i = 0; i < P; ++i) {
        if (anc[i] < 0 || anc[i] >= P) { bad = 1; continue; }
        off[anc[i]] += 1;
    }
    return bad ? ORACLE_FLAG_BAD_ANCESTOR : 0;
}

/* Inverse direction: particle j repeated o_j times, in index order. */
int oracle_offspring_to_ancestors(const int32_t *off, int32_t *anc, int64_t P)
{
    if (!anc || !off || P < 1) return ORACLE_EINVAL;
    int64_t i = 0;
    for (int64_t j = 0; j < P; ++j)
        for (int32_t c = 0; c < off[j]; ++c) {
            if (i >= P) return ORACLE_EINVAL;
            anc[i++] = (int32_t)j;
        }
    return i == P ? 0 : ORACLE_EINVAL;
}

int oracle_permute_copy(const int32_t *anc, const float *x_in, float *x_out, int64_t P, int32_t D)
{
    if (!anc || !x_in || !x_out || P < 1 || D < 1) return ORACLE_EINVAL;
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
    for (int64_t i = 0; i < P; ++i) {
        if (anc[i] < 0 || anc[i] >= P) { bad = 1; continue; }
        memcpy(x_out + i * (int64_t)D, x_in + (int64_t)anc[i] * D, (size_t)D * sizeof(float));
    }
    return bad ? ORACLE_FLAG_BAD_ANCESTOR : 0;
}

/*
 * Minimal-copy state update from offspring counts (Sec. 2 gives the output
 * of a resampler as offspring o_j, the number of copies of particle j in the
 * new population, and says converting between offspring and ancestors is
 * straightforward). After resampling every particle carries weight 1 / P,
 * so the new population is defined by its multiset {x_j repeated o_j times};
 * the slot order is free. This update keeps every row j with o_j >= 1 in its
 * own slot and fills each empty slot (o_i = 0) with one of the extra copies
 * (o_j - 1 of them for each j with o_j >= 2): the holes in increasing slot
 * order take the extras in increasing order of j. A source j is never a
 * hole, so the update can be done in place. anc_out[i] is the particle whose
 * row slot i holds afterwards. Counts that are negative or do not sum to P
 * leave x unchanged, anc_out the identity, and return the bad-ancestor flag.
 */
int oracle_offspring_update_inplace(const int32_t *off, float *x, int64_t P, int32_t D,
                                    int32_t *anc_out)
{
    if (!off || !x || !anc_out || P < 1 || D < 1) return ORACLE_EINVAL;
    int64_t total = 0;
    for (int64_t j = 0; j < P; ++j) {
        if (off[j] < 0) total = -1;
        if (total >= 0) total += off[j];
    }
    for (int64_t i = 0; i < P; ++i) anc_out[i] = (int32_t)i;
    if (total != P) return ORACLE_FLAG_BAD_ANCESTOR;
    /* walk the holes and the extra copies together, both in increasing order */
    int64_t j = 0;     /* current source particle */
    int32_t used = 0;  /* extra copies of j already placed */
    for (int64_t i = 0; i < P; ++i) {
        if (off[i] != 0) continue;
        while (j < P && off[j] - 1 - used <= 0) {  /* no extra copy of j left */
            ++j;
            used = 0;
        }
        if (j >= P) return ORACLE_EINVAL;  /* not reached when the counts sum to P */
        anc_out[i] = (int32_t)j;
        memcpy(x + i * (int64_t)D, x + j * (int64_t)D, (size_t)D * sizeof(float));
        ++used;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Number of Metropolis iterations B (Sec. 2, eqs. (1)-(5)): the two-state   */
/* chain Z_n on "is the chain at p_max" has alpha = (1 - w_max) / (P w_max), */
/* beta = 1 / P, lambda = 1 - alpha - beta, and the deviation of             */
/* P(Z_B = 1 | Z_0) from w_max is at most epsilon once                       */
/* B >= log(eps (alpha + beta) / max(alpha, beta)) / log(lambda).            */
/* w_max is the normalised largest weight. Returns the smallest integer      */
/* B >= 0 with lambda^B <= eps (alpha + beta) / max(alpha, beta) (eq. (4));  */
/* eq. (5) is that inequality solved for 0 < lambda < 1. At lambda = 0       */
/* (uniform weights) eq. (4) needs B = 1: one step reaches stationarity.     */
/* P = 1 needs no iterations.                                                */
/* ------------------------------------------------------------------------ */

uint32_t oracle_metropolis_B(int64_t P, double w_max, double eps)
{
    if (P < 2 || !(w_max > 0.0) || w_max > 1.0 || !(eps > 0.0)) return 0;
    double alpha = (1.0 - w_max) / ((double)P * w_max);
    double beta = 1.0 / (double)P;
    double lambda = 1.0 - alpha - beta;
    double target = eps * (alpha + beta) / (alpha > beta ? alpha : beta);
    if (target >= 1.0) return 0;
    if (!(lambda > 0.0)) return 1;
    double b = ceil(log(target) / log(lambda));
    if (b < 0.0) return 0;
    if (b > 4294967295.0) return 4294967295u;
    return (uint32_t)b;
}

/* ------------------------------------------------------------------------ */
/* Accuracy of one resampling (Sec. 3, Fig. 2 caption):                      */
/* sum_i (o_i / P - w_i / W)^2 with w_i = exp(lw_i - m), W = sum_j w_j.      */
/* ------------------------------------------------------------------------ */

double oracle_resampling_error(const int32_t *off, const float *lw, int64_t P)
{
    if (!off || !lw || P < 1) return NAN;
    double *C = (double *)malloc((size_t)P * sizeof(double));
    float m = 0.0f;
    if (!C) return NAN;
    if (oracle_cumulative(lw, P, C, &m, NULL) != 0) {
        free(C);
        return NAN;
    }
    double W = C[P - 1];
    double err = 0.0;
    for (int64_t i = 0; i < P; ++i) {
        double p = exp((double)lw[i] - (double)m) / W;
        double e = (double)off[i] / (double)P - p;
        err += e * e;
    }
    free(C);
    return err;
}

/* ------------------------------------------------------------------------ */
/* Bootstrap particle filter (Sec. 1: initialisation, propagation,           */
/* weighting, resampling) for the linear-Gaussian model                      */
/*   x_0 ~ N(0, I),  x_t = A x_{t-1} + N(0, q I),  y_t = x_t + N(0, r I).    */
/* The proposal is the transition, so the weight is the observation density. */
/* Gaussian noise: Box-Muller on Philox block (i, t, h, 5), h = 0..ceil(D/4)-1 */
/* giving components 4h..4h+3: (r0, r1) -> z_{4h}, z_{4h+1} and              */
/* (r2, r3) -> z_{4h+2}, z_{4h+3}, with u1 = (r + 1/2) 2^-32, u2 = r' 2^-32, */
/* z = sqrt(-2 log u1) (cos, sin)(2 pi u2). Time 0 draws the initial state.  */
/* ------------------------------------------------------------------------ */

static void filter_normals(uint64_t seed, int64_t i, uint32_t t, int32_t D, double *z)
{
    const double two_pi = 6.283185307179586476925286766559;
    for (int32_t h = 0; 4 * h < D; ++h) {
        uint32_t r[4];
        draw_block(seed, (uint32_t)i, t, (uint32_t)h, TAG_FILTER_NOISE, r);
        for (int pair = 0; pair < 2; ++pair) {
            double u1 = ((double)r[2 * pair] + 0.5) * 0x1p-32;
            double u2 = (double)r[2 * pair + 1] * 0x1p-32;
            double rad = sqrt(-2.0 * log(u1));
            int d0 = 4 * h + 2 * pair;
            if (d0 < D) z[d0] = rad * cos(two_pi * u2);
            if (d0 + 1 < D) z[d0 + 1] = rad * sin(two_pi * u2);
        }
    }
}

/* Initial state: x_0^i = z(i, t = 0). Row-major [P x D] binary32. */
int oracle_filter_init(float *x, int64_t P, int32_t D, uint64_t seed)
{
    if (!x || P < 1 || D < 1 || D > 64) return ORACLE_EINVAL;
    double z[64];
    for (int64_t i = 0; i < P; ++i) {
        filter_normals(seed, i, 0, D, z);
        for (int32_t d = 0; d < D; ++d) x[i * D + d] = (float)z[d];
    }
    return 0;
}

/* One propagate + weight step at time t >= 1: x_out = A x_in + sqrt(q) z,   */
/* lw = log N(y_t; x_out, r I). A is row-major [D x D] binary64.             */
int oracle_filter_step(const float *x_in, float *x_out, float *lw, int64_t P, int32_t D,
                       const double *A, const float *y, double q, double r, uint64_t seed,
                       uint32_t t)
{
    if (!x_in || !x_out || !lw || !A || !y || P < 1 || D < 1 || D > 64) return ORACLE_EINVAL;
    const double log_two_pi = 1.8378770664093454835606594728112;
    double z[64];
    double sq = sqrt(q);
    double norm = -0.5 * (double)D * (log_two_pi + log(r));
    for (int64_t i = 0; i < P; ++i) {
        filter_normals(seed, i, t, D, z);
        double ss = 0.0;
        for (int32_t a = 0; a < D; ++a) {
            double acc = 0.0;
            for (int32_t b = 0; b < D; ++b) acc += A[a * D + b] * (double)x_in[i * D + b];
            float xa = (float)(acc + sq * z[a]);
            x_out[i * D + a] = xa;
            double e = (double)y[a] - (double)xa;
            ss += e * e;
        }
        lw[i] = (float)(norm - 0.5 * ss / r);
    }
    return 0;
}

/* Full filter over t = 1..T. resampler: 0 stratified, 1 Metropolis(B).     */
/* Resampling at time t uses instance t. Returns the log-likelihood estimate */
/* sum_t [ log(sum_i exp(lw_i)) - log P ] in *loglik.                        */
int oracle_bootstrap_filter(const double *A, const float *y, int32_t T, int32_t D, int64_t P,
                            double q, double r, uint64_t seed, int resampler, uint32_t B,
                            double *loglik, float *x_final)
{
    if (!A || !y || !loglik || T < 0 || P < 1 || D < 1 || D > 64) return ORACLE_EINVAL;
    float *x = (float *)malloc((size_t)P * D * sizeof(float));
    float *xp = (float *)malloc((size_t)P * D * sizeof(float));
    float *lw = (float *)malloc((size_t)P * sizeof(float));
    double *C = (double *)malloc((size_t)P * sizeof(double));
    int32_t *anc = (int32_t *)malloc((size_t)P * sizeof(int32_t));
    int rc = 0;
    if (!x || !xp || !lw || !C || !anc) { rc = ORACLE_EINVAL; goto done; }
    oracle_filter_init(x, P, D, seed);
    double ll = 0.0;
    for (int32_t t = 1; t <= T; ++t) {
        oracle_filter_step(x, xp, lw, P, D, A, y + (int64_t)(t - 1) * D, q, r, seed, (uint32_t)t);
        float m = 0.0f;
        if (oracle_cumulative(lw, P, C, &m, NULL) != 0) { rc = ORACLE_EINVAL; goto done; }
        ll += (double)m + log(C[P - 1]) - log((double)P);
        if (resampler == 0) rc = oracle_stratified(lw, anc, P, seed, (uint32_t)t, NULL, NULL);
        else rc = oracle_metropolis(lw, anc, P, B, seed, (uint32_t)t, NULL);
        if (rc != 0) goto done;
        oracle_permute_copy(anc, xp, x, P, D);
    }
    *loglik = ll;
    if (x_final) memcpy(x_final, x, (size_t)P * D * sizeof(float));
done:
    free(x); free(xp); free(lw); free(C); free(anc);
    return rc;
}
