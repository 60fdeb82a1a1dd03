"""Particle MCMC over batched filters on the GPU.

  - run 0 of the batched filters equals K single bootstrap filters (keys
    seed + k, variances q_k): the same particles bit for bit and the same
    log-likelihood estimates up to the order of the float64 sums;
  - the estimates scatter around the Kalman log-likelihood (unbiased in Z,
    so log Z-hat sits below log Z by about half its variance);
  - particle marginal Metropolis-Hastings over log q lands on the posterior
    computed on a grid from the Kalman likelihood.
"""
import math

import numpy as np
import pytest
import torch

from oracle.kalman import kalman_loglik
from paper_1202_6163_amd import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def model():
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    A = workloads.filter_model(D=4, seed=1)
    y = workloads.filter_observations(A, T=30, q=0.1, r=0.5, seed=3)
    return A, y


def test_batched_filters_equal_single_filters(model):
    from paper_1202_6163_amd.filter import BootstrapFilter
    from paper_1202_6163_amd.pmcmc import BatchedFilters
    A, y = model
    K, P = 5, 3000
    q = np.array([0.05, 0.1, 0.2, 0.1, 0.4])
    bf = BatchedFilters(A, K, P, r=0.5, seed=70)
    yd = torch.from_numpy(y).cuda()
    ll = bf.loglik(q, yd, run=0)
    assert int(bf.status.sum()) == 0
    for k in range(K):
        one = BootstrapFilter(A, P, q=q[k], r=0.5, seed=70 + k, resampler="stratified")
        llk = one.run(y)
        assert abs(ll[k] - llk) < 1e-9 * max(1.0, abs(llk)), (k, ll[k], llk)
        assert torch.equal(bf.x[k * P:(k + 1) * P].view(torch.int32), one.x.view(torch.int32))


def test_batched_estimates_scatter_around_kalman(model):
    from paper_1202_6163_amd.pmcmc import BatchedFilters
    A, y = model
    K, P = 64, 4096
    bf = BatchedFilters(A, K, P, r=0.5, seed=5)
    ll = bf.loglik(np.full(K, 0.1), torch.from_numpy(y).cuda(), run=0)
    exact = kalman_loglik(A, y, 0.1, 0.5)
    sd = ll.std(ddof=1)
    # E[log Z-hat] ~ log Z - var/2; allow four standard errors around that
    assert abs(ll.mean() - (exact - 0.5 * sd * sd)) < 4 * sd / math.sqrt(K) + 1e-3, (
        ll.mean(), exact, sd)
    # runs draw fresh numbers
    ll2 = bf.loglik(np.full(K, 0.1), torch.from_numpy(y).cuda(), run=1)
    assert not np.array_equal(ll, ll2)


def test_pmmh_recovers_grid_posterior(model):
    from paper_1202_6163_amd.pmcmc import BatchedFilters, pmmh
    A, y = model
    prior_mean, prior_sd = math.log(0.1), 1.0
    grid = np.linspace(math.log(0.01), math.log(1.0), 241)
    logpost = np.array([kalman_loglik(A, y, math.exp(g), 0.5) for g in grid])
    logpost += -0.5 * ((grid - prior_mean) / prior_sd) ** 2
    w = np.exp(logpost - logpost.max())
    w /= w.sum()
    post_mean = float((w * grid).sum())
    post_sd = float(math.sqrt((w * (grid - post_mean) ** 2).sum()))
    K, P = 64, 2048
    bf = BatchedFilters(A, K, P, r=0.5, seed=11)
    chain, rate = pmmh(bf, torch.from_numpy(y).cuda(), iters=80, theta0=math.log(0.1),
                       step=0.5 * post_sd * 2.38, prior_mean=prior_mean, prior_sd=prior_sd,
                       seed=2)
    samples = chain[30:].ravel()
    print(f"PMMH mean {samples.mean():.3f} sd {samples.std():.3f} accept {rate:.2f}; "
          f"grid posterior mean {post_mean:.3f} sd {post_sd:.3f}")
    assert 0.05 < rate < 0.95
    assert abs(samples.mean() - post_mean) < 0.35 * post_sd
    assert 0.5 * post_sd < samples.std() < 1.6 * post_sd
