"""Host logic of the particle-MCMC driver (CPU): the Metropolis-Hastings
decision per chain with a log-likelihood estimate in place of the
likelihood (Sec. 1's motivating use of the particle filter)."""
import math

import numpy as np

from paper_1202_6163_amd.pmcmc import accept_step, log_prior


def test_better_proposals_always_accept_and_nan_never():
    theta = np.zeros(4)
    ll = np.array([-10.0, -10.0, -10.0, -10.0])
    prop = np.zeros(4)
    ll_prop = np.array([-5.0, -10.0, np.nan, -np.inf])
    u = np.full(4, 0.999999)
    th, l2, acc = accept_step(theta, ll, prop, ll_prop, u, 0.0, 1.0)
    # equal log-likelihoods give log alpha = 0 > log u: accepted too
    assert acc.tolist() == [True, True, False, False]
    assert l2[0] == -5.0 and l2[2] == -10.0


def test_acceptance_rate_matches_exp_log_alpha():
    rng = np.random.default_rng(0)
    n = 200_000
    theta = np.zeros(n)
    prop = np.zeros(n)
    ll = np.zeros(n)
    ll_prop = np.full(n, math.log(0.3))
    _, _, acc = accept_step(theta, ll, prop, ll_prop, rng.random(n), 0.0, 1.0)
    assert abs(acc.mean() - 0.3) < 5 * math.sqrt(0.3 * 0.7 / n)


def test_prior_enters_the_ratio():
    theta = np.array([0.0])
    prop = np.array([1.0])
    # equal likelihoods: the ratio is the prior ratio exp(-1/2) under N(0, 1)
    rng = np.random.default_rng(1)
    n = 100_000
    _, _, acc = accept_step(np.zeros(n), np.zeros(n), np.ones(n), np.zeros(n), rng.random(n),
                            0.0, 1.0)
    assert abs(acc.mean() - math.exp(-0.5)) < 0.01
    assert log_prior(prop, 0.0, 1.0)[0] - log_prior(theta, 0.0, 1.0)[0] == -0.5
