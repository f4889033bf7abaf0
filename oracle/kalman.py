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


def kalman_means(x0, observations, q: float, r: float) -> np.ndarray:
    """Posterior means of (x, y, vx, vy) after each observation.

    x0: the initial state (x, y, vx, vy), known exactly (zero covariance).
    observations: [K][2] observed positions.
    Returns [K][4] means.
    """
    Fm = np.array([[1.0, 1.0], [0.0, 1.0]])
    Qm = q * np.array([[1.0 / 3.0, 0.5], [0.5, 1.0]])
    H = np.array([[1.0, 0.0]])
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
