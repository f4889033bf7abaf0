"""The oracle's record of ambiguous patch centres, and the per-PE and master
steps it reruns for another valid choice of centre (used by the GPU parity
tests, which take the centre the GPU chose where both are valid).

The likelihood at the other centre is checked against a brute-force sum over
the patch written here (the Gaussian log-likelihood ratio of Sec. V's spot
model); the rerun per-PE and master steps against the trace of an ordinary
iteration and against their closed forms (log-sum-exp, weighted mean).
"""
import numpy as np
import pytest

import oracle.oracle as orc
from paper_1310_4624_amd import synth
from tests import helpers as H


def brute_patch_loglik(frame, x, y, I, cx, cy, half=4, s=1.5, B=5.0, sn=2.0):
    Hh, W = frame.shape
    if not (-half <= cx <= W - 1 + half and -half <= cy <= Hh - 1 + half):
        return 0.0
    acc = 0.0
    for v in range(int(cy) - half, int(cy) + half + 1):
        for u in range(int(cx) - half, int(cx) + half + 1):
            if 0 <= u < W and 0 <= v < Hh:
                g = np.exp(-((u - x) ** 2 + (v - y) ** 2) / (2 * s * s))
                r0 = float(frame[v, u]) - B
                acc += (r0 * r0 - (r0 - I * g) ** 2) / (2 * sn * sn)
    return acc


def case(eps_abs):
    cfg = dict(n_filters=2, n_pe=3, n_per_pe=100, width=40, height=36, mode=1, seed=5,
               patch=9, psf_sigma=1.5, background=5.0, noise_sigma=2.0)
    rng = np.random.Generator(np.random.PCG64(3))
    truth = np.array([[[15.3, 20.7, 0, 0, 12.0], [36.6, 3.2, 0, 0, 9.0]]])
    frame = synth.render(truth[0], 40, 36, 1.5, 5.0, 2.0, rng)
    state = synth.random_state(rng, 2, 3, 100, 40, 36, spread=1.5, centre=truth[0, :, :2],
                               I0=10.0)
    L = rng.normal(0, 3, (2, 3))
    o = orc.Oracle(cfg, np.zeros((2, 5), np.float32))
    o.set_state(state.astype(np.float64), L, 4)
    o.set_ambiguity(0.0, eps_abs)
    return cfg, frame, o.step(frame)


def test_ambiguity_mask_and_alternative_likelihoods():
    eps = 0.05
    cfg, frame, tr = case(eps)
    x, y, I = tr["prop"][0], tr["prop"][1], tr["prop"][4]
    for bit, c in ((1, x), (2, y)):
        t = c + 0.5
        want = np.abs(t - np.floor(t + 0.5)) <= eps
        assert np.array_equal((tr["amb"] & bit) != 0, want)
    assert 20 < np.count_nonzero(tr["amb"]) < 200
    ox, oy = H.other_centre(x), H.other_centre(y)
    fx, fy = np.floor(x + 0.5), np.floor(y + 0.5)
    for g in np.flatnonzero(tr["amb"]):
        a = tr["amb"][g]
        assert tr["ell"][g] == pytest.approx(
            brute_patch_loglik(frame, x[g], y[g], I[g], fx[g], fy[g]), rel=1e-9, abs=1e-9)
        alts = [(1, ox[g], fy[g]), (2, fx[g], oy[g]), (3, ox[g], oy[g])]
        for j, (need, cx, cy) in enumerate(alts):
            if (a & need) == need:
                assert abs(cx - fx[g]) + abs(cy - fy[g]) >= 1
                want = brute_patch_loglik(frame, x[g], y[g], I[g], cx, cy)
                assert tr["ell_alt"][g, j] == pytest.approx(want, rel=1e-9, abs=1e-9)
            else:
                assert np.isnan(tr["ell_alt"][g, j])


def test_ambiguity_does_not_change_the_iteration():
    _, _, a = case(0.05)
    _, _, b = case(0.0)
    for key in ("ell", "Q", "anc", "L_pe", "xhat", "n_ex_next", "state"):
        assert np.array_equal(a[key], b[key]), key


def test_rerun_with_other_centres():
    """Take the other centre for every ambiguous particle: select_branches
    reruns steps 6-10 with those likelihoods; the PE masses are log-sum-exps of
    lambda + l and the estimates weighted means (closed forms), and PEs
    without a change keep the trace values."""
    cfg, frame, tr = case(0.05)
    F, M, n_p = 2, 3, 100
    cand = np.concatenate([tr["ell"][:, None], tr["ell_alt"]], axis=1)
    pick = np.where(np.isfinite(cand[:, 3]), 3, np.where(np.isfinite(cand[:, 1]), 1,
                                                          np.where(np.isfinite(cand[:, 2]), 2, 0)))
    ell_gpu = cand[np.arange(len(pick)), pick]
    tol = H.coord_tol(tr["prop"][0])
    ref, tl, chosen = H.select_branches(cfg, frame, tr, ell_gpu, H.ell_tolerance,
                                        (tol, tol, tol), 5)
    assert np.array_equal(chosen, pick)
    assert np.array_equal(ref["ell"], ell_gpu)
    for pe in range(F * M):
        f, m = divmod(pe, M)
        sl = slice(pe * n_p, (pe + 1) * n_p)
        u = tr["lambda"][sl] + ell_gpu[sl]
        assert ref["L_pe"][f, m] == pytest.approx(np.logaddexp.reduce(u), rel=1e-12, abs=1e-12)
        w = np.exp(u - u.max())
        assert np.allclose(ref["xhat_pe"][f, m], (tr["prop"][:, sl] * w).sum(1) / w.sum(),
                           rtol=1e-12, atol=1e-12)
        if not pick[sl].any():
            assert np.array_equal(ref["Q"][sl], tr["Q"][sl])
            assert ref["L_pe"][f, m] == tr["L_pe"][f, m]
    for f in range(F):
        Lg = np.logaddexp.reduce(ref["L_pe"][f])
        assert ref["L_glob"][f] == pytest.approx(Lg, rel=1e-12)
        assert ref["log_z"][f] == pytest.approx(Lg - np.log(n_p), rel=1e-12)
        wm = np.exp(ref["L_pe"][f] - Lg)
        assert np.allclose(ref["xhat"][f], (wm[:, None] * ref["xhat_pe"][f]).sum(0), atol=1e-12)
