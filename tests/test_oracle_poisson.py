"""Pins of the oracle's Poisson likelihood (photon-count pixels, the noise of
the paper's synthetic images, Fig. 1).

l = sum over the patch of log p(z | B + I g) - log p(z | B) for Poisson
pixels; checked against SciPy's Poisson log-pmf (an independent
implementation), against the maximum of the expected log-likelihood at the
true state, and through the whole filter on a Poisson sequence.
"""
import numpy as np
import pytest
from scipy import stats

from oracle import oracle as O
from paper_1310_4624_amd import synth


def _cfg(**over):
    return synth.filter_config("rna_128_4x256_poisson", **over)


def _brute(cfg, frame, st):
    x, y, I = st[0], st[1], st[4]
    half = cfg["patch"] // 2
    H, W = frame.shape
    B, s2 = float(np.float32(cfg["background"])), float(np.float32(cfg["psf_sigma"])) ** 2
    cx, cy = int(np.floor(x + 0.5)), int(np.floor(y + 0.5))
    tot = 0.0
    for v in range(cy - half, cy + half + 1):
        for u in range(cx - half, cx + half + 1):
            if not (0 <= u < W and 0 <= v < H):
                continue
            g = np.exp(-((u - x) ** 2 + (v - y) ** 2) / (2 * s2))
            z = int(frame[v, u])
            tot += stats.poisson.logpmf(z, B + I * g) - stats.poisson.logpmf(z, B)
    return tot


def test_poisson_ratio_matches_scipy_logpmf():
    cfg = _cfg(width=40, height=30)
    rng = np.random.Generator(np.random.PCG64(11))
    frame = synth.render_poisson(np.array([[12.3, 14.6, 0, 0, 25.0]]), 40, 30, 1.5, 10.0, rng)
    pts = np.concatenate([rng.uniform(-3, 42, (40, 2)), [[0.2, 0.4], [39.6, 29.4], [-4.2, 5.0]]])
    for x, y in pts:
        st = np.array([x, y, 0.3, -0.2, rng.uniform(5, 40)])
        got = O.loglik(cfg, frame, 0, st)
        assert got == pytest.approx(_brute(cfg, frame, st), rel=1e-10, abs=1e-9)


def test_expected_counts_maximum_at_truth():
    """With the expected counts as data, E[l(x)] = sum lam log(1 + I g_x / B) -
    I g_x is maximal at the true state (Gibbs' inequality pixel by pixel)."""
    cfg = _cfg(width=32, height=32)
    xt, yt, It = 15.2, 16.1, 20.0
    ys, xs = np.mgrid[0:32, 0:32].astype(np.float64)
    lam = 10.0 + It * np.exp(-((xs - xt) ** 2 + (ys - yt) ** 2) / (2 * 1.5 ** 2))
    frame = lam.astype(np.float32)
    best = O.loglik(cfg, frame, 0, np.array([xt, yt, 0, 0, It]))
    for dx in np.linspace(-0.3, 0.3, 7):
        for dy in np.linspace(-0.3, 0.3, 7):
            for dI in (-2.0, 0.0, 2.0):
                if dx == dy == dI == 0.0:
                    continue
                v = O.loglik(cfg, frame, 0, np.array([xt + dx, yt + dy, 0, 0, It + dI]))
                assert v < best + 1e-6, (dx, dy, dI)


def test_filter_tracks_poisson_spot():
    wl = "rna_128_4x256_poisson"
    cfg = synth.filter_config(wl, seed=5)
    seq = synth.make_sequence(wl, seed=1000)
    o = O.Oracle(cfg, seq.initial_truth())
    err = []
    for k in range(1, seq.frames.shape[0] + 1):
        tr = o.step(seq.frames[k - 1], want={"xhat"})
        err.append(np.sum((tr["xhat"][0, :2] - seq.truth[k, 0, :2]) ** 2))
    assert np.sqrt(np.mean(err)) < 0.5
