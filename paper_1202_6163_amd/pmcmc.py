"""Particle marginal Metropolis-Hastings with K filters run as one batch.

Sec. 1 of the paper motivates fast resampling by particle MCMC, which runs a
whole particle filter for every parameter proposal. Here K Markov chains
over the state-noise variance q of the linear-Gaussian model
    x_0 ~ N(0, I),  x_t = A x_{t-1} + N(0, q I),  y_t = x_t + N(0, r I)
advance together: every iteration proposes log q'_k = log q_k + s z_k for
each chain, runs the K filters at once (one batched propagate+weight launch
and one batched resampling per time step, the plan replayed with a fresh
Philox instance word per step and run), accumulates each filter's log
likelihood estimate on the device, and accepts or rejects each chain on the
host with the estimate in place of the likelihood. The prior is
log q ~ N(prior_mean, prior_sd^2).

Filter k of run 0 computes exactly what BootstrapFilter(seed = seed + k,
q = q_k) computes; later runs draw fresh numbers (another initial key, time
words shifted by run (T + 1)).
"""
import math

import numpy as np
import torch

from . import api
from .batch import Batch


class BatchedFilters:
    def __init__(self, A, K, P, r=0.5, seed=0, resampler="stratified", device=None):
        if resampler not in ("stratified", "systematic"):
            raise ValueError("batched filters resample with 'stratified' or 'systematic'")
        self.device = torch.device(device) if device is not None else torch.device(
            "cuda", torch.cuda.current_device())
        dev = self.device
        self.A = torch.as_tensor(A, dtype=torch.float64).contiguous().to(dev)
        self.D = int(self.A.shape[0])
        self.K, self.P, self.r, self.seed = int(K), int(P), float(r), int(seed)
        KP = self.K * self.P
        self.x = torch.empty((KP, self.D), dtype=torch.float32, device=dev)
        self.xp = torch.empty_like(self.x)
        self.lw = torch.empty(KP, dtype=torch.float32, device=dev)
        self.anc = torch.empty(KP, dtype=torch.int32, device=dev)
        self.status = torch.zeros(self.K, dtype=torch.int32, device=dev)
        self.q = torch.zeros(self.K, dtype=torch.float64, device=dev)
        self.acc = torch.zeros(self.K, dtype=torch.float64, device=dev)
        insts = []
        for k in range(self.K):
            rows = slice(k * self.P, (k + 1) * self.P)
            insts.append(dict(lw=self.lw[rows], anc=self.anc[rows], kind=resampler,
                              seed=self.seed + k, instance=0, x_in=self.xp[rows],
                              x_out=self.x[rows], status=self.status[k:k + 1]))
        self.batch = Batch(insts, device=dev)

    def loglik(self, q, y, run=0):
        """Log-likelihood estimates of the K filters for variances q[K] on
        observations y[T, D] (a float32 device tensor); one host sync."""
        T = int(y.shape[0])
        self.q.copy_(torch.as_tensor(np.asarray(q, dtype=np.float64)))
        self.acc.zero_()
        base = run * (T + 1)  # time words of this run: base + 1 .. base + T
        api.filter_init_batch(self.x, self.K, self.seed + run * self.K)
        for t in range(1, T + 1):
            api.filter_propagate_weight_batch(self.x, self.A, y[t - 1], self.q, self.r, self.seed,
                                              base + t, self.K, self.xp, self.lw)
            self.batch.run(instance_add=base + t)
            self.batch.add_log_mean_weight(self.acc)
        return self.acc.cpu().numpy()


def log_prior(theta, mean, sd):
    return -0.5 * ((theta - mean) / sd) ** 2


def accept_step(theta, ll, proposal, ll_prop, u, prior_mean, prior_sd):
    """One Metropolis-Hastings decision per chain (symmetric random walk on
    log q): accept iff log u < (ll' + prior') - (ll + prior). A NaN
    log-likelihood of the proposal never accepts. Returns (theta, ll, accepted)."""
    log_alpha = (ll_prop + log_prior(proposal, prior_mean, prior_sd)) - (
        ll + log_prior(theta, prior_mean, prior_sd))
    acc = np.log(u) < np.nan_to_num(log_alpha, nan=-np.inf)
    return np.where(acc, proposal, theta), np.where(acc, ll_prop, ll), acc


def pmmh(filters, y, iters, theta0, step=0.3, prior_mean=math.log(0.1), prior_sd=1.0, seed=0):
    """K chains of particle marginal Metropolis-Hastings over theta = log q.
    Returns (chain[iters + 1, K] of theta, acceptance rate)."""
    rng = np.random.default_rng(seed)
    theta = np.broadcast_to(np.asarray(theta0, dtype=np.float64), (filters.K,)).copy()
    ll = filters.loglik(np.exp(theta), y, run=0)
    chain = [theta.copy()]
    accepted = 0
    for it in range(1, iters + 1):
        prop = theta + step * rng.standard_normal(filters.K)
        ll_prop = filters.loglik(np.exp(prop), y, run=it)
        theta, ll, acc = accept_step(theta, ll, prop, ll_prop, rng.random(filters.K), prior_mean,
                                     prior_sd)
        accepted += int(acc.sum())
        chain.append(theta.copy())
    return np.array(chain), accepted / (iters * filters.K)
