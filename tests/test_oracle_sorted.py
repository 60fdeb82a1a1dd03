"""Pins for the oracle's sorted-weight variants (CPU only).

Sec. 3 compares the resamplers with and without sorting the weights before
the prefix sum (sorting makes the multinomial bisection faster; the paper
finds it not worth its cost). A sorted variant runs the resampler on the
weights in decreasing order and maps the ancestors back. Pins:
  - the order against a brute-force comparison sort, with ties, -inf, +-0;
  - already-decreasing weights: the variant equals the plain resampler;
  - relabelling the particles relabels the ancestors draw for draw;
  - systematic floor/ceil bounds and unbiasedness still hold (any order);
  - the multinomial error keeps its closed-form mean (order-free).
"""
import numpy as np
import pytest
from scipy import stats

import oracle
from paper_1202_6163_amd import workloads

KINDS = ["stratified", "systematic", "multinomial"]
PLAIN = {"stratified": oracle.stratified, "systematic": oracle.systematic,
         "multinomial": oracle.multinomial}


def probs(lw):
    w = np.exp(lw.astype(np.float64) - lw.max())
    return w / w.sum()


def test_order_brute_force():
    rng = np.random.default_rng(3)
    for trial in range(200):
        n = int(rng.integers(1, 40))
        vals = np.array([0.0, -0.0, 1.5, -2.0, -np.inf, 3.25], dtype=np.float32)
        lw = rng.choice(vals, size=n).astype(np.float32)
        if trial % 2:
            lw = rng.standard_normal(n).astype(np.float32)
        want = sorted(range(n), key=lambda i: (-(float(lw[i]) + 0.0), i))
        assert list(oracle.sorted_order(lw)) == want


@pytest.mark.parametrize("kind", KINDS)
def test_decreasing_input_is_unchanged(kind):
    lw = np.sort(workloads.normal_logweights(3000, 1.0, 5))[::-1].copy()
    a, st = oracle.sorted_variant(kind, lw, 7, 1)
    b, st2 = PLAIN[kind](lw, 7, 1)
    assert st == st2 == 0 and np.array_equal(a, b)


@pytest.mark.parametrize("kind", KINDS)
def test_relabelling_relabels_ancestors(kind):
    P = 2500
    lw = workloads.normal_logweights(P, 2.0, 9)
    assert np.unique(lw).size == P  # distinct weights: the order is unique
    perm = np.random.default_rng(1).permutation(P).astype(np.int32)
    a, _ = oracle.sorted_variant(kind, lw, 4, 0)
    a2, _ = oracle.sorted_variant(kind, lw[perm], 4, 0)
    assert np.array_equal(perm[a2], a)


def test_flags_give_identity():
    lw = np.zeros(100, dtype=np.float32)
    lw[7] = np.nan
    a, st = oracle.sorted_variant("multinomial", lw, 1)
    assert st == oracle.FLAG_NAN and np.array_equal(a, np.arange(100))


def test_systematic_bounds_any_order():
    P = 1024
    lw = workloads.normal_logweights(P, 1.5, 2)
    e = P * probs(lw)
    for s in range(10):
        a, _ = oracle.sorted_variant("systematic", lw, s)
        off = np.bincount(a, minlength=P)
        assert off.sum() == P
        assert np.all(off >= np.floor(e - 1e-9)) and np.all(off <= np.ceil(e + 1e-9))


@pytest.mark.slow
@pytest.mark.parametrize("kind", KINDS)
def test_unbiased(kind):
    P, R = 48, 3000
    lw = workloads.normal_logweights(P, 1.0, 31)
    e = P * probs(lw)
    offs = np.empty((R, P))
    for s in range(R):
        a, _ = oracle.sorted_variant(kind, lw, s, 3)
        offs[s] = np.bincount(a, minlength=P)
    mean, se = offs.mean(0), offs.std(0, ddof=1) / np.sqrt(R)
    nz = se > 0
    assert np.allclose(mean[~nz], e[~nz], atol=1e-9)
    chi2 = (((mean[nz] - e[nz]) / se[nz]) ** 2).sum()
    assert stats.chi2.sf(chi2, int(nz.sum())) >= 1e-4


@pytest.mark.slow
def test_multinomial_error_closed_form():
    P, R = 512, 300
    lw = workloads.normal_logweights(P, 1.0, 30)
    p = probs(lw)
    err = []
    for s in range(R):
        a, _ = oracle.sorted_variant("multinomial", lw, s)
        off, _ = oracle.ancestors_to_offspring(a)
        err.append(oracle.resampling_error(off, lw))
    err = np.array(err)
    expect = (1.0 - (p ** 2).sum()) / P
    assert abs(err.mean() - expect) < 4.5 * err.std(ddof=1) / np.sqrt(R)
