"""Textbook Kalman filter for the linear-Gaussian special case of the tracker.

TEST INFRASTRUCTURE ONLY (part of the oracle; see oracle.py).

With point observations z_k = (x_k, y_k) + N(0, r I) and the nearly-constant-
velocity dynamics of the benchmark (per axis F = [[1, 1], [0, 1]],
Q = q [[1/3, 1/2], [1/2, 1]]), the posterior of Eq. 1-2 is Gaussian and its mean
is given exactly by the Kalman recursion.  A particle filter run on the same
model converges to that mean as the number of particles grows.
"""
from __future__ import annotations

import numpy as np

_F = np.array([[1.0, 1.0], [0.0, 1.0]])
_H = np.array([[1.0, 0.0]])


def _q(q: float) -> np.ndarray:
    return q * np.array([[1.0 / 3.0, 0.5], [0.5, 1.0]])


def kalman_means(x0, observations, q: float, r: float) -> np.ndarray:
    """Posterior means of (x, y, vx, vy) after each observation.

    x0: the initial state (x, y, vx, vy), known exactly (zero covariance).
    observations: [K][2] observed positions.
    Returns [K][4] means.
    """
    Fm, Qm, H = _F, _q(q), _H
    out = np.zeros((len(observations), 4))
    for axis, (pi, vi) in enumerate(((0, 2), (1, 3))):
        m = np.array([x0[pi], x0[vi]], dtype=np.float64)
        P = np.zeros((2, 2))
        for k, z in enumerate(observations):
            m = Fm @ m
            P = Fm @ P @ Fm.T + Qm
            S = (H @ P @ H.T)[0, 0] + r
            K = (P @ H.T)[:, 0] / S
            m = m + K * (z[axis] - m[0])
            P = P - np.outer(K, H @ P)
            out[k, pi] = m[0]
            out[k, vi] = m[1]
    return out


def kalman_log_marginal(x0, observations, q: float, r: float) -> np.ndarray:
    """log p(z_k | z_1..z_{k-1}) for k = 1..K, the normalization of Eq. 1 in the
    linear-Gaussian case: the predictive density of z_k is Gaussian with mean
    H m_k^- and variance S_k = H P_k^- H^T + r per axis (the two axes are
    independent), so the increment is the sum over the axes of
    -(z - H m^-)^2 / (2 S) - log(2 pi S) / 2.

    x0: the initial state (x, y, vx, vy), known exactly (zero covariance).
    Returns [K] increments.
    """
    Fm, Qm, H = _F, _q(q), _H
    out = np.zeros(len(observations))
    for pi, vi in ((0, 2), (1, 3)):
        m = np.array([x0[pi], x0[vi]], dtype=np.float64)
        P = np.zeros((2, 2))
        for k, z in enumerate(observations):
            m = Fm @ m
            P = Fm @ P @ Fm.T + Qm
            S = (H @ P @ H.T)[0, 0] + r
            innov = z[0 if pi == 0 else 1] - m[0]
            out[k] += -0.5 * innov * innov / S - 0.5 * np.log(2.0 * np.pi * S)
            K = (P @ H.T)[:, 0] / S
            m = m + K * innov
            P = P - np.outer(K, H @ P)
    return out
