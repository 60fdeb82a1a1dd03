"""Pins for the oracle's prefix-sum resamplers (CPU only).

Sec. 2 (Fig. 1(a-c)): multinomial places P independent uniform arrows on the
weight circle, stratified one uniform arrow per stratum [i/P, (i+1)/P),
systematic the same offset in every stratum; all read the ancestor off the
cumulative weights. Pins:
  - cumulative sums: exact for equal weights, within the binary64 summation
    bound of an 80-bit extended-precision sum otherwise;
  - the search rule against a brute-force scan;
  - equal weights give the identity (stratified, systematic) and i.i.d.
    uniform ancestors (multinomial, chi-square);
  - systematic offspring in {floor(P w_i/W), ceil(P w_i/W)}, stratified
    offspring within 2 of P w_i/W, offspring summing to P;
  - unbiasedness E[o_i] = P w_i / W by Monte Carlo;
  - the multinomial error's closed-form mean (1 - sum p^2) / P and the
    ordering stratified <= multinomial (Sec. 3).
"""
import numpy as np
import pytest
from scipy import stats

import oracle
from paper_1202_6163_amd import workloads

RESAMPLERS = {"stratified": oracle.stratified, "systematic": oracle.systematic,
              "multinomial": oracle.multinomial}


def probs(lw):
    w = np.exp(lw.astype(np.float64) - lw.max())
    return w / w.sum()


def test_cumulative_equal_weights_exact():
    for P in (1, 7, 1024, 100_000):
        C, m, st = oracle.cumulative(np.full(P, -3.5, dtype=np.float32))
        assert st == 0 and m == np.float32(-3.5)
        assert np.array_equal(C, np.arange(1, P + 1, dtype=np.float64))


@pytest.mark.parametrize("sigma", [0.25, 1.0, 4.0])
def test_cumulative_within_summation_bound(sigma):
    P = 1 << 16
    lw = workloads.normal_logweights(P, sigma, seed=4)
    C, m, st = oracle.cumulative(lw)
    hi, lo = oracle.cumulative_extended(lw)
    ref = hi + lo
    n = np.arange(1, P + 1)
    # left-to-right binary64 sum of positive terms, each exp within 1 ulp
    bound = (n + 1) * 2.0**-52
    rel = np.abs(C - ref) / ref
    assert np.all(rel <= bound)
    assert m == lw.max()
    assert np.all(np.diff(C) >= 0)


def test_cumulative_negative_infinity_contributes_zero():
    lw = np.array([0.0, -np.inf, 1.0, -np.inf], dtype=np.float32)
    C, _, st = oracle.cumulative(lw)
    assert st == 0
    assert C[1] == C[0] and C[3] == C[2] and C[2] == 1.0 + np.exp(-1.0)


def test_flags():
    lw = np.zeros(8, dtype=np.float32)
    lw[2] = np.nan
    assert oracle.cumulative(lw)[2] == oracle.FLAG_NAN
    lw[2] = np.inf
    assert oracle.cumulative(lw)[2] == oracle.FLAG_POSINF
    lw[:] = -np.inf
    assert oracle.cumulative(lw)[2] == oracle.FLAG_ALL_NEGINF
    anc, st = oracle.stratified(lw, 1)
    assert st == oracle.FLAG_ALL_NEGINF and np.array_equal(anc, np.arange(8))


def brute_search(C, x):
    W = C[-1]
    if x < W:
        return int(np.flatnonzero(C > x)[0])
    return int(np.flatnonzero(C == W)[0])


def test_search_rule_brute_force():
    rng = np.random.default_rng(0)
    lw = rng.standard_normal(64).astype(np.float32)
    lw[[0, 5, 6, 63]] = -np.inf  # zero weights at both ends and inside
    C, _, _ = oracle.cumulative(lw)
    xs = list(rng.random(500) * C[-1]) + list(C) + [0.0, C[-1], C[-1] * 1.5, np.nextafter(C[-1], 0)]
    for x in xs:
        j = oracle.search(C, x)
        assert j == brute_search(C, x)
        assert np.isfinite(lw[j])  # a zero-weight particle is never selected


@pytest.mark.parametrize("P", [1, 2, 1000, 4096, 65537])
def test_equal_weights_identity(P):
    lw = np.zeros(P, dtype=np.float32)
    for name in ("stratified", "systematic"):
        anc, st = RESAMPLERS[name](lw, seed=7, instance=3)
        assert st == 0 and np.array_equal(anc, np.arange(P)), name


def test_multinomial_equal_weights_uniform():
    P, R = 50, 2000
    lw = np.zeros(P, dtype=np.float32)
    counts = np.zeros(P)
    for s in range(R):
        anc, _ = oracle.multinomial(lw, seed=s)
        counts += np.bincount(anc, minlength=P)
    chi2 = ((counts - R) ** 2 / R).sum()
    assert stats.chi2.sf(chi2, P - 1) >= 1e-4


def test_multinomial_chi_square_against_weights():
    P, R = 40, 2500
    lw = workloads.normal_logweights(P, 1.0, seed=8)
    p = probs(lw)
    counts = np.zeros(P)
    for s in range(R):
        anc, _ = oracle.multinomial(lw, seed=s, instance=1)
        counts += np.bincount(anc, minlength=P)
    expect = P * R * p
    chi2 = ((counts - expect) ** 2 / expect).sum()
    assert stats.chi2.sf(chi2, P - 1) >= 1e-4


@pytest.mark.parametrize("sigma", [0.5, 2.0, 4.0])
def test_offspring_bounds(sigma):
    P = 2048
    lw = workloads.normal_logweights(P, sigma, seed=12)
    e = P * probs(lw)
    for s in range(20):
        anc, _ = oracle.systematic(lw, seed=s)
        off, rc = oracle.ancestors_to_offspring(anc)
        assert rc == 0 and off.sum() == P
        assert np.all(np.diff(anc) >= 0)  # sorted ancestors
        assert np.all(off >= np.floor(e - 1e-9)) and np.all(off <= np.ceil(e + 1e-9))
        anc, _ = oracle.stratified(lw, seed=s)
        off, _ = oracle.ancestors_to_offspring(anc)
        assert off.sum() == P and np.all(np.diff(anc) >= 0)
        assert np.all(np.abs(off - e) < 2.0)


@pytest.mark.slow
@pytest.mark.parametrize("name", ["stratified", "systematic", "multinomial"])
def test_unbiased_offspring(name):
    P, R = 64, 3000
    lw = workloads.normal_logweights(P, 1.0, seed=21)
    e = P * probs(lw)
    offs = np.empty((R, P))
    for s in range(R):
        anc, _ = RESAMPLERS[name](lw, seed=s, instance=2)
        offs[s] = np.bincount(anc, minlength=P)
    mean = offs.mean(0)
    se = offs.std(0, ddof=1) / np.sqrt(R)
    nz = se > 0
    # particles with zero variance must be exactly at their expectation
    assert np.allclose(mean[~nz], e[~nz], atol=1e-9)
    z = (mean[nz] - e[nz]) / se[nz]
    chi2 = (z**2).sum()
    assert stats.chi2.sf(chi2, int(nz.sum())) >= 1e-4


@pytest.mark.slow
def test_error_ordering_and_multinomial_closed_form():
    P, R = 512, 300
    lw = workloads.normal_logweights(P, 1.0, seed=30)
    p = probs(lw)
    err = {k: [] for k in RESAMPLERS}
    for s in range(R):
        for name, fn in RESAMPLERS.items():
            anc, _ = fn(lw, seed=s)
            off, _ = oracle.ancestors_to_offspring(anc)
            err[name].append(oracle.resampling_error(off, lw))
    e_mult = np.array(err["multinomial"])
    expect = (1.0 - (p**2).sum()) / P
    assert abs(e_mult.mean() - expect) < 4.5 * e_mult.std(ddof=1) / np.sqrt(R)
    assert np.mean(err["stratified"]) < e_mult.mean()
    assert np.mean(err["systematic"]) < e_mult.mean()


def test_draw_points_strata():
    P, W = 4096, 123.25
    x = oracle.draw_points(oracle.KIND_STRATIFIED, P, W, seed=5, instance=1)
    d = W / P
    i = np.arange(P)
    assert np.all(x >= i * d) and np.all(x < (i + 1) * d)
    U = x / d - i
    assert stats.kstest(U, "uniform").pvalue >= 1e-4
    xs = oracle.draw_points(oracle.KIND_SYSTEMATIC, P, W, seed=5, instance=1)
    off = xs - i * d
    assert np.all(off >= 0) and np.all(off < d) and np.ptp(off) < 1e-9
    xm = oracle.draw_points(oracle.KIND_MULTINOMIAL, P, W, seed=5, instance=1)
    assert np.all(xm >= 0) and np.all(xm < W)
    assert stats.kstest(xm / W, "uniform").pvalue >= 1e-4
    # different instances draw different points
    x2 = oracle.draw_points(oracle.KIND_STRATIFIED, P, W, seed=5, instance=2)
    assert np.mean(x2 == x) < 0.01


def test_cumw_output_matches_cumulative():
    lw = workloads.normal_logweights(3000, 2.0, seed=2)
    C, _, _ = oracle.cumulative(lw)
    for name, fn in RESAMPLERS.items():
        anc, st, Cw = fn(lw, seed=1, want_cumw=True)
        assert np.array_equal(Cw, C)
        x = oracle.draw_points({"stratified": 0, "systematic": 1, "multinomial": 2}[name],
                               lw.size, C[-1], seed=1)
        want = np.array([brute_search(C, v) for v in x[:300]])
        assert np.array_equal(anc[:300], want)
