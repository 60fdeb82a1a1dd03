"""Pins for the oracle's Metropolis resampler (CPU only).

Sec. 2 of the paper defines the Metropolis resampler as P independent chains,
each proposing an index uniformly over all P particles and accepting by the
weight ratio, and analyses B through a two-state chain (eqs. (1)-(5)). These
tests pin the oracle to:
  - B = 0 gives the identity (each chain starts at its own index);
  - equal weights accept every proposal, so a_i is the last proposal;
  - a single finite weight is reached with probability 1 - (1 - 1/P)^B;
  - for P <= 6 the law of a_i is row i of the exact B-step transition matrix
    (chi-square over 10^6 resamplings; threshold p >= 1e-4);
  - the two-state lumping of that matrix equals the paper's closed form.

The acceptance probabilities use the exact discrete law of the binary32 u
grid: #{u : L(u) < d} / 2^23 with L from an 80-bit logarithm.
"""
import numpy as np
import pytest
from scipy import stats

import oracle


@pytest.fixture(scope="module")
def L_sorted():
    m = np.arange(1 << 23, dtype=np.int64)
    u = ((2 * m + 1) * 2.0**-24).astype(np.float32)
    L = np.log(u.astype(np.longdouble)).astype(np.float32)
    return np.sort(L)


def accept_prob(L_sorted, d):
    """P(L(u) < d) on the u grid, d a binary32 value (NaN never accepts)."""
    d = np.float32(d)
    if np.isnan(d):
        return 0.0
    return np.searchsorted(L_sorted, d, side="left") / float(1 << 23)


def proposal_probs(P):
    """Exact probability of each index under j = floor(r P / 2^32)."""
    j = np.arange(P + 1, dtype=object)
    edges = [-(-(int(v) << 32) // P) for v in j]  # ceil(j 2^32 / P)
    return np.array([(edges[k + 1] - edges[k]) / 2.0**32 for k in range(P)])


def metropolis_matrix(lw, L_sorted):
    lw = np.asarray(lw, dtype=np.float32)
    P = lw.size
    q = proposal_probs(P)
    M = np.zeros((P, P))
    for k in range(P):
        for j in range(P):
            if j != k:
                with np.errstate(invalid="ignore"):
                    d = np.float32(lw[j] - lw[k])
                M[k, j] = q[j] * accept_prob(L_sorted, d)
        M[k, k] = 1.0 - M[k].sum()
    return M


def test_B_zero_is_identity():
    lw = np.random.default_rng(0).standard_normal(257).astype(np.float32)
    anc, st = oracle.metropolis(lw, 0, seed=3)
    assert st == 0
    assert np.array_equal(anc, np.arange(257))


def test_equal_weights_accept_every_proposal():
    P, B, seed, inst = 1000, 7, 11, 5
    lw = np.full(P, 1.25, dtype=np.float32)
    anc, _ = oracle.metropolis(lw, B, seed, inst)
    n = B - 1
    key = [seed & 0xFFFFFFFF, seed >> 32]
    for i in range(P):
        r = oracle.philox4x32_10([i, inst, n // 2, 1], key)
        j = oracle.index(int(r[2] if n % 2 else r[0]), P)
        assert anc[i] == j


def test_single_finite_weight_hit_probability():
    P, B, p = 8, 5, 3
    lw = np.full(P, -np.inf, dtype=np.float32)
    lw[p] = -2.0
    n_inst = 40000
    anc = oracle.metropolis_many(lw, B, 17, 0, n_inst)
    assert np.all(anc[:, p] == p)  # the chain at the finite weight never leaves
    others = np.delete(anc, p, axis=1)
    # a chain at -inf accepts the finite proposal and rejects every other one
    assert np.all((others == p) | (others == np.delete(np.arange(P), p)[None, :]))
    hit = (others == p).mean()
    expect = 1.0 - (1.0 - 1.0 / P) ** B
    n = others.size
    z = (hit - expect) / np.sqrt(expect * (1 - expect) / n)
    # chains within one instance are independent; |z| < 4.4 has p >= 1e-5
    assert abs(z) < 4.4, (hit, expect)


CASES = [
    (np.array([0.0, -1.0, 0.5, -2.5], dtype=np.float32), 3, 101),
    (np.random.default_rng(5).standard_normal(6).astype(np.float32), 8, 102),
    (np.array([0.3, -np.inf, -0.7], dtype=np.float32), 5, 103),
    (np.array([1.0, 1.0, -0.5, 2.0, 1.0], dtype=np.float32), 4, 104),
    (np.array([0.0, 0.0], dtype=np.float32), 1, 105),
]


@pytest.mark.slow
@pytest.mark.parametrize("lw,B,seed", CASES)
def test_exact_law_small_P(lw, B, seed, L_sorted):
    P = lw.size
    M = metropolis_matrix(lw, L_sorted)
    MB = np.linalg.matrix_power(M, B)
    n_inst = 1_000_000 if P <= 4 else 400_000
    anc = oracle.metropolis_many(lw, B, seed, 0, n_inst)
    chi2, dof = 0.0, 0
    for i in range(P):
        counts = np.bincount(anc[:, i], minlength=P)
        expect = n_inst * MB[i]
        zero = expect < 1e-12
        assert np.all(counts[zero] == 0), (i, counts, expect)
        chi2 += ((counts[~zero] - expect[~zero]) ** 2 / expect[~zero]).sum()
        dof += int((~zero).sum()) - 1
    pval = stats.chi2.sf(chi2, dof)
    # false-failure rate of this threshold: 1e-4 per case
    assert pval >= 1e-4, (chi2, dof, pval)


def test_two_state_lumping_matches_closed_form():
    # Eqs. (1)-(3): with continuous acceptance min(1, w_j / w_k) the chain
    # "at p_max or not" is exactly Markov with alpha = (1 - w_max) / (P w_max)
    # and beta = 1 / P, so M^B[p_max, p_max] = (beta + alpha lambda^B) / (alpha + beta).
    rng = np.random.default_rng(9)
    for P in (3, 6, 17):
        w = rng.gamma(1.0, size=P)
        w /= w.sum()
        M = np.zeros((P, P))
        for k in range(P):
            for j in range(P):
                if j != k:
                    M[k, j] = min(1.0, w[j] / w[k]) / P
            M[k, k] = 1.0 - M[k].sum()
        pm = int(np.argmax(w))
        wm = w[pm]
        a, b = (1 - wm) / (P * wm), 1.0 / P
        lam = 1 - a - b
        for B in (1, 2, 5, 20, 40):
            MB = np.linalg.matrix_power(M, B)
            assert abs(MB[pm, pm] - (b + a * lam**B) / (a + b)) < 1e-13
            for k in range(P):
                if k != pm:
                    assert abs(MB[k, pm] - b * (1 - lam**B) / (a + b)) < 1e-13


def test_status_flags_nan_posinf():
    lw = np.zeros(16, dtype=np.float32)
    lw[3] = np.nan
    _, st = oracle.metropolis(lw, 4, 1)
    assert st == oracle.FLAG_NAN
    lw[3] = np.inf
    _, st = oracle.metropolis(lw, 4, 1)
    assert st == oracle.FLAG_POSINF
    lw[:] = -np.inf
    anc, st = oracle.metropolis(lw, 9, 1)
    assert st == 0 and np.array_equal(anc, np.arange(16))  # all -inf: every move rejected


@pytest.mark.slow
def test_converged_error_matches_multinomial():
    # Sec. 3: once converged, the Metropolis resampler's error matches the
    # multinomial resampler's, whose expectation is (1 - sum p_i^2) / P.
    P = 256
    lw = np.random.default_rng(2).standard_normal(P).astype(np.float32) * np.float32(0.5)
    w = np.exp(lw.astype(np.float64) - lw.max())
    p = w / w.sum()
    expect = (1.0 - (p**2).sum()) / P
    R = 400
    errs = []
    for s in range(R):
        anc, _ = oracle.metropolis(lw, 64, seed=1000 + s)
        off, _ = oracle.ancestors_to_offspring(anc)
        errs.append(oracle.resampling_error(off, lw))
    errs = np.array(errs)
    se = errs.std(ddof=1) / np.sqrt(R)
    assert abs(errs.mean() - expect) < 4.5 * se, (errs.mean(), expect, se)
