"""Kalman-filter closed form of the log-likelihood (test infrastructure only).

For the linear-Gaussian model used by the bootstrap-filter harness,
    x_0 ~ N(0, I),  x_t = A x_{t-1} + N(0, q I),  y_t = x_t + N(0, r I),
the marginal likelihood p(y_{1:T}) is available exactly; a bootstrap particle
filter (Sec. 1: initialisation, propagation, weighting, resampling) estimates
it without bias, so the filter's estimate must agree with it within Monte
Carlo error. Computed in binary64 with numpy.
"""
import numpy as np


def kalman_loglik(A, y, q, r):
    A = np.asarray(A, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    T, D = y.shape
    I = np.eye(D)
    mean = np.zeros(D)
    cov = np.eye(D)
    ll = 0.0
    for t in range(T):
        mean = A @ mean
        cov = A @ cov @ A.T + q * I
        S = cov + r * I
        resid = y[t] - mean
        sign, logdet = np.linalg.slogdet(S)
        assert sign > 0
        sol = np.linalg.solve(S, resid)
        ll += -0.5 * (D * np.log(2.0 * np.pi) + logdet + resid @ sol)
        K = np.linalg.solve(S, cov).T  # cov S^-1 (S and cov symmetric)
        mean = mean + K @ resid
        cov = (I - K) @ cov
        cov = 0.5 * (cov + cov.T)
    return float(ll)
