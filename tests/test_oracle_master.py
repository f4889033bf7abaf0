"""Pins of the oracle's master step (Alg. 3 steps 9-10): the log-likelihood
increment log p(z_k | z_1..z_{k-1}) and PE_eff (Eq. 4), traced through whole
iterations of ``orc_step``.

* In the linear-Gaussian special case (point observations, NCV dynamics) the
  exact increment is the Kalman predictive density; the filter's estimate
  converges to it as the number of particles grows.
* With identical particles and no process noise every PE's mass is a closed
  form of the carried masses, so PE_eff, the next N_ex and the increment are
  known exactly (integers and rational arithmetic on the test side).
"""
import math
from fractions import Fraction

import numpy as np
import pytest
from scipy.stats import multivariate_normal

import oracle.oracle as orc
from oracle.kalman import kalman_log_marginal
from paper_1310_4624_amd import synth


# ------------------------------------------------ the Kalman reference itself
def joint_gaussian_log_marginal(x0, obs, q, r):
    """log p(z_1..z_K) from the joint Gaussian of the observations of one axis
    pair, built directly from the linear model (no recursion): with
    x_k = F^k x0 + sum_{l<=k} F^{k-l} w_l and z_k = H x_k + v_k,
    Cov(z_i, z_j) = H (sum_{l<=min(i,j)} F^{i-l} Q F^{j-l}^T) H^T + r [i=j]."""
    K = len(obs)
    Fm = np.array([[1.0, 1.0], [0.0, 1.0]])
    Qm = q * np.array([[1.0 / 3.0, 0.5], [0.5, 1.0]])
    Fp = [np.linalg.matrix_power(Fm, n) for n in range(K + 1)]
    total = 0.0
    for pi, vi in ((0, 2), (1, 3)):
        m0 = np.array([x0[pi], x0[vi]])
        mean = np.array([(Fp[k] @ m0)[0] for k in range(1, K + 1)])
        C = np.zeros((K, K))
        for i in range(1, K + 1):
            for j in range(1, K + 1):
                acc = np.zeros((2, 2))
                for l in range(1, min(i, j) + 1):
                    acc += Fp[i - l] @ Qm @ Fp[j - l].T
                C[i - 1, j - 1] = acc[0, 0] + (r if i == j else 0.0)
        total += multivariate_normal(mean, C).logpdf(obs[:, 0 if pi == 0 else 1])
    return total


def test_kalman_increments_sum_to_joint_gaussian():
    truth, obs = synth.point_sequence(5, 3, 7, q=0.5, r=1.0)
    for f in range(3):
        inc = kalman_log_marginal(truth[0, f, :4], obs[:, f].astype(np.float64), 0.5, 1.0)
        want = joint_gaussian_log_marginal(truth[0, f, :4], obs[:, f].astype(np.float64), 0.5, 1.0)
        assert inc.sum() == pytest.approx(want, rel=1e-10, abs=1e-9)


# ---------------------------------- log p(z_k | z_1..z_{k-1}) vs the Kalman value
@pytest.mark.parametrize("mode,ratio", [(orc.MODE_RNA, 0.0), (orc.MODE_RNA, 0.1),
                                        (orc.MODE_RNA, 0.5), (orc.MODE_ARNA, 0.1)])
def test_log_z_converges_to_kalman_marginal(mode, ratio):
    """Sum over 8 frames of the traced increment, plus the Gaussian constant
    -log(2 pi r) that the point likelihood leaves out, against the exact log
    marginal likelihood.  A dropped -log N_p, -log M in its place or a
    missing renormalization by W_{k-1} moves the sum by tens of nats."""
    F, K, q, r = 6, 8, 0.5, 1.0
    truth, obs = synth.point_sequence(21, F, K, q=q, r=r)
    t32 = truth[0].astype(np.float32)
    kf = np.array([kalman_log_marginal(t32[f, :4].astype(np.float64),
                                       obs[:, f].astype(np.float64), float(np.float32(q)),
                                       float(np.float32(r))) for f in range(F)])
    mean_abs = {}
    for logn in (12, 16):
        M = 4
        cfg = dict(n_filters=F, n_pe=M, n_per_pe=(1 << logn) // M, width=128, height=128,
                   mode=mode, lik_mode=orc.LIK_POINT, fixed_ratio=ratio, initial_ratio=0.1,
                   q=q, noise_sigma=math.sqrt(r), sigma_I=0.5, seed=1000 + logn)
        o = orc.Oracle(cfg, t32)
        inc = np.zeros((F, K))
        for k in range(K):
            inc[:, k] = o.step(obs[k], want={"log_z"})["log_z"] - math.log(2 * math.pi * r)
        err = inc - kf
        mean_abs[logn] = float(np.abs(err.sum(axis=1)).mean())
        if logn == 16:
            assert np.all(np.abs(err) < 0.1), np.abs(err).max()
            assert np.all(np.abs(err.sum(axis=1)) < 0.2), err.sum(axis=1)
    assert mean_abs[16] < mean_abs[12], mean_abs


# ------------------------------------------- closed forms with identical particles
def identical_particle_step(L_prev, n_p=64, mode=orc.MODE_RNA, ratio=0.0):
    """One iteration from M PEs of identical particles (x0 moving with v, no
    process noise), carried log masses L_prev, point observation z."""
    M = len(L_prev)
    x0 = np.array([40.25, 31.5, 0.75, -0.5, 6.0])
    z = np.array([[41.5, 30.25]], np.float32)
    cfg = dict(n_filters=1, n_pe=M, n_per_pe=n_p, width=64, height=64, mode=mode,
               lik_mode=orc.LIK_POINT, fixed_ratio=ratio, initial_ratio=ratio, eff_cutoff=0.99,
               q=0.0, sigma_I=0.0, noise_sigma=1.5, seed=99)
    o = orc.Oracle(cfg, x0[None].astype(np.float32))
    state = np.repeat(x0[:, None], M * n_p, axis=1)
    o.set_state(state, np.asarray(L_prev, np.float64)[None], 5)
    tr = o.step(z, want={"pe_eff", "log_z", "P", "n_ex", "n_ex_next", "xhat", "L_pe", "L_glob",
                         "ring_pred"})
    x1 = x0[:2] + x0[2:4]
    s2 = float(np.float32(1.5)) ** 2
    ell = -float(np.sum((x1 - z[0].astype(np.float64)) ** 2)) / (2 * s2)
    return tr, ell, x1


def eq3_nex(P, n_p, cutoff_ppm=990000):
    """Eq. 3 with PE_eff = S^2 / D in exact rational arithmetic."""
    M = len(P)
    S = sum(int(p) for p in P)
    D = sum(int(p) * int(p) for p in P)
    if M == 1:
        return 0
    if D == 0:
        return n_p // 2
    if Fraction(S * S, M * D) > Fraction(cutoff_ppm, 1000000):
        return 0
    return math.floor(Fraction(n_p * (M * D - S * S), 2 * (M - 1) * D))


@pytest.mark.parametrize("M", [1, 2, 5, 64])
def test_pe_eff_equal_masses_is_m(M):
    tr, ell, x1 = identical_particle_step(np.full(M, -3.0))
    assert tr["pe_eff"][0] == M
    assert np.all(tr["P"] == 1 << 20)
    assert tr["n_ex_next"][0] == 0   # RNA at 0%
    assert tr["log_z"][0] == pytest.approx(ell, abs=1e-9)
    assert np.allclose(tr["xhat"][0, :2], x1, atol=1e-12)


@pytest.mark.parametrize("k,M", [(1, 8), (3, 8), (5, 16), (7, 7)])
def test_pe_eff_k_equal_masses_is_k(k, M):
    """k PEs with equal mass, the others dead (-inf): PE_eff = k; k = 1 is
    'one PE holds all the mass'."""
    L = np.full(M, -np.inf)
    L[np.arange(k) * (M // k)] = 1.7
    tr, ell, _ = identical_particle_step(L)
    assert tr["pe_eff"][0] == k
    assert np.count_nonzero(tr["P"]) == k
    # the carried masses sum to one after renormalization: the increment is
    # the likelihood of the (single) particle position
    assert tr["log_z"][0] == pytest.approx(ell, abs=1e-9)


def safe_floor(x):
    """floor of positive values that lie at least 0.01 from an integer (or
    are exactly 2^20), else None: rounding of order 1e-13 cannot move them."""
    frac = x - np.floor(x)
    ok = ((frac > 0.01) & (frac < 0.99)) | (x == 2.0 ** 20)
    return np.floor(x).astype(np.int64) if np.all(ok) else None


def test_pe_eff_of_unequal_masses_exact():
    """RNA-0%: after the step every PE mass is its carried mass times the same
    factor, so P_m = floor(exp(L_m - max L) 2^20) is known from L_prev, and
    PE_eff = S^2 / D exactly."""
    rng = np.random.Generator(np.random.PCG64(77))
    for trial in range(6):
        M = int(rng.integers(2, 40))
        P = None
        while P is None:
            L = rng.normal(0.0, 1.5, M)
            P = safe_floor(np.exp(L - L.max()) * 2.0 ** 20)
        tr, ell, _ = identical_particle_step(L)
        assert np.array_equal(tr["P"][0].astype(np.int64), P), trial
        S, D = int(P.sum()), int((P * P).sum())
        assert tr["pe_eff"][0] == pytest.approx(float(Fraction(S * S, D)), rel=1e-14)
        assert tr["log_z"][0] == pytest.approx(ell, abs=1e-9)
        # the renormalized carried masses sum to one: L_glob = ell + log N_p
        assert tr["L_glob"][0] == pytest.approx(ell + math.log(64), abs=1e-9)


def test_arna_exchange_and_next_nex_exact():
    """ARNA with unequal carried masses: this iteration's N_ex is Eq. 3 of the
    carried masses; after the exchange PE m holds N_p - N_ex particles of its
    own mass and N_ex of pred(m)'s, so its new mass is proportional to
    (N_p - N_ex) W_m + N_ex W_pred(m); PE_eff and the next N_ex follow."""
    rng = np.random.Generator(np.random.PCG64(78))
    n_p, done = 64, 0
    while done < 6:
        M = int(rng.integers(3, 30))
        L = rng.normal(0.0, 1.0, M)
        P_prev = safe_floor(np.exp(L - L.max()) * 2.0 ** 20)
        if P_prev is None:
            continue
        nex = eq3_nex(P_prev, n_p)
        if nex == 0:
            continue
        tr, ell, _ = identical_particle_step(L, n_p=n_p, mode=orc.MODE_ARNA, ratio=0.1)
        assert tr["n_ex"][0] == nex
        pred = tr["ring_pred"][0].astype(np.int64)
        W = (n_p - nex) * np.exp(L - L.max()) + nex * np.exp(L[pred] - L.max())
        P = safe_floor(W / W.max() * 2.0 ** 20)
        if P is None:
            continue
        assert np.array_equal(tr["P"][0].astype(np.int64), P)
        S, D = int(P.sum()), int((P * P).sum())
        assert tr["pe_eff"][0] == pytest.approx(float(Fraction(S * S, D)), rel=1e-14)
        assert tr["n_ex_next"][0] == eq3_nex(P, n_p)
        assert tr["log_z"][0] == pytest.approx(ell, abs=1e-9)
        done += 1
