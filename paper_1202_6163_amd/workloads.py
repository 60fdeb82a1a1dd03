"""Seeded synthetic inputs for the resampling stage.

This module only draws input data (log-weights, particle state, model
matrices, observation sequences, request streams). It holds none of the
resampling arithmetic, imports neither the oracle nor the HIP library, and is
the one module both sides share. Every generator is a pure function of its
seed.

Shapes follow the paper's experiments (Sec. 3): weight sets of P particles with
a swept spread. The paper draws Dirichlet(alpha) weights; the headline sweep
uses i.i.d. normal log-weights lw = sigma * z, whose effective sample size
e^{-sigma^2} P spans the same range (sigma = 0.31, 0.83, 1.55, 2.15 match the
ESS of alpha = 10, 1, .1, .01). ``dirichlet_logweights`` gives the paper's own
weight sets.
"""
import math

import numpy as np

SIGMAS = (0.25, 0.5, 1.0, 2.0, 4.0)
SWEEP_P = tuple(1 << k for k in (12, 14, 16, 18, 20))
SWEEP_B = (8, 16, 32, 64, 128, 256, 512)


def normal_logweights(P, sigma, seed):
    """lw = sigma * z, z ~ N(0,1) binary32 from numpy's default_rng(seed).

    For sigma a power of two the product is exact in binary32.
    """
    z = np.random.default_rng(seed).standard_normal(int(P), dtype=np.float32)
    return (np.float32(sigma) * z).astype(np.float32)


def small_case_logweights():
    """The small single-resample case: P = 1024, lw ~ N(0, 1), seed 1."""
    return np.random.default_rng(1).standard_normal(1024, dtype=np.float32)


def dirichlet_logweights(P, alpha, seed):
    """log w for w ~ Dirichlet(alpha, ..., alpha), unnormalised.

    Gamma(alpha) variates underflow for small alpha, so their logarithms are
    drawn as log G(alpha + 1) + log(U) / alpha.
    """
    rng = np.random.default_rng(seed)
    g = rng.gamma(alpha + 1.0, size=int(P))
    u = rng.random(int(P))
    return (np.log(g) + np.log(u) / alpha).astype(np.float32)


def state_rows_exact(P, D):
    """State rows that identify themselves: X[i, d] = i + d / 8 (exact for i < 2^21)."""
    i = np.arange(int(P), dtype=np.float64)[:, None]
    d = np.arange(int(D), dtype=np.float64)[None, :]
    return (i + d / 8.0).astype(np.float32)


def state_rows_normal(P, D, seed):
    return np.random.default_rng(seed).standard_normal((int(P), int(D)), dtype=np.float32)


# ----------------------------------------------------------------- filter model
def filter_model(D=8, seed=0, skew_norm=0.05):
    """A = 0.95 I + S with S skew-symmetric of spectral norm skew_norm."""
    rng = np.random.default_rng(seed)
    G = rng.standard_normal((D, D))
    S = G - G.T
    S *= skew_norm / np.linalg.norm(S, 2)
    return 0.95 * np.eye(D) + S


def filter_observations(A, T, q=0.1, r=0.5, seed=0):
    """Simulate x_0 ~ N(0, I), x_t = A x_{t-1} + N(0, qI), y_t = x_t + N(0, rI)."""
    A = np.asarray(A, dtype=np.float64)
    D = A.shape[0]
    rng = np.random.default_rng(1000 + seed)
    x = rng.standard_normal(D)
    ys = np.empty((int(T), D))
    for t in range(int(T)):
        x = A @ x + math.sqrt(q) * rng.standard_normal(D)
        ys[t] = x + math.sqrt(r) * rng.standard_normal(D)
    return ys.astype(np.float32)


# ----------------------------------------------------------------- batched
def batch_instances(n=1024, seed=0, p_lo=8, p_hi=16, s_lo=0.25, s_hi=3.0):
    """Instance sizes P_k = floor(2^(p_lo + (p_hi - p_lo) v)) and spreads sigma_k."""
    rng = np.random.default_rng(seed)
    v = rng.random(int(n))
    P = np.floor(np.exp2(p_lo + (p_hi - p_lo) * v)).astype(np.int64)
    sig = rng.uniform(s_lo, s_hi, size=int(n))
    return P, sig


def batch_logweights(P, sig, seed=0):
    """Concatenated log-weights of all instances (float32), and their offsets."""
    offs = np.zeros(len(P) + 1, dtype=np.int64)
    offs[1:] = np.cumsum(P)
    rng = np.random.default_rng(seed + 1)
    lw = np.empty(int(offs[-1]), dtype=np.float32)
    for k in range(len(P)):
        z = rng.standard_normal(int(P[k]), dtype=np.float32)
        lw[offs[k]:offs[k + 1]] = (np.float32(sig[k]) * z)
    return lw, offs


# ----------------------------------------------------------------- serving
SERVE_SLOTS = 16      # client payload slots
SERVE_SIGMA = (0.5, 4.0)


def serve_slot_sigma(k, n_slots=SERVE_SLOTS, s_lo=SERVE_SIGMA[0], s_hi=SERVE_SIGMA[1]):
    """The weight spread of payload slot k: the slots cover [s_lo, s_hi] evenly."""
    return s_lo + (s_hi - s_lo) * (k + 0.5) / n_slots


def serve_payload(k, p_max=1 << 20):
    """Payload slot k: (lw[p_max] = sigma_k z, x[p_max * 16] standard normal)."""
    rng = np.random.default_rng(7000 + k)
    z = rng.standard_normal(int(p_max), dtype=np.float32)
    lw = (np.float32(serve_slot_sigma(k)) * z).astype(np.float32)
    x = rng.standard_normal(int(p_max) * 16, dtype=np.float32)
    return lw, x


# Requests with weights this even use the Metropolis resampler; the rest
# stratified or systematic. Sec. 3 finds Metropolis competitive only when the
# weights vary little: above this spread eq. (5)'s B at 2^20 particles
# exceeds a thousand iterations (sigma = 1: B = 257), where the prefix-sum
# resamplers are faster.
SERVE_METROPOLIS_MAX_SIGMA = 1.1


def request_stream(rate=2000.0, duration=60.0, seed=0, p_lo=10, p_hi=20, dims=(1, 16), B=64,
                   n_slots=SERVE_SLOTS):
    """Poisson arrivals: list of dicts (t_arrival s, P, sigma, slot, D, kind, B, seed).
    A request's data lives in payload slot `slot` (uniform over the slots), so
    its sigma is that slot's: uniform over SERVE_SIGMA in n_slots steps. The
    client picks the resampler from its weights' spread: Metropolis up to
    SERVE_METROPOLIS_MAX_SIGMA, otherwise stratified or systematic."""
    rng = np.random.default_rng(seed)
    n_max = int(rate * duration * 1.2 + 100)
    gaps = rng.exponential(1.0 / rate, size=n_max)
    t = np.cumsum(gaps)
    n = int(np.searchsorted(t, duration))
    t = t[:n]
    P = np.floor(np.exp2(p_lo + (p_hi - p_lo) * rng.random(n))).astype(np.int64)
    slot = rng.integers(0, n_slots, size=n)
    D = rng.choice(np.asarray(dims), size=n)
    prefix = rng.choice(np.asarray(["stratified", "systematic"]), size=n)
    sig = [serve_slot_sigma(int(slot[k]), n_slots) for k in range(n)]
    kind = ["metropolis" if sig[k] <= SERVE_METROPOLIS_MAX_SIGMA else str(prefix[k])
            for k in range(n)]
    return [dict(id=k, t=float(t[k]), P=int(P[k]), sigma=sig[k], slot=int(slot[k]), D=int(D[k]),
                 kind=kind[k], B=int(B), seed=int(k)) for k in range(n)]
