"""Pins of the oracle's gradient of the log marginal likelihood.

The objective is the filter's own estimate J = sum_k log Zhat_k of
log p(z_1..z_K) (steps 9-10 of Alg. 3 with the step-4 renormalization), with
the discrete choices of the run held fixed.  The oracle differentiates it in
forward mode; these tests pin that derivative to central finite differences
of an independent re-evaluation of J with the recorded choices, and pin the
re-evaluation itself to the ordinary filter step.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1310_4624_amd import synth

CASES = {
    # plain RNA, fixed ring, one spot
    "rna": dict(wl="rna_128_4x256", over={}, frames=8),
    # ARNA with the adaptive ratio, two filters, tracking start
    "arna": dict(wl="rna_128_4x256",
                 over=dict(mode=O.MODE_ARNA, n_filters=2, n_pe=8, n_per_pe=128), frames=8),
    # ARNA from the information-sharing start (large exchanges, spread PEs)
    "infoshare": dict(wl="rna_128_4x256",
                      over=dict(mode=O.MODE_ARNA, init_mode=O.INIT_INFOSHARE, n_pe=6,
                                n_per_pe=256), frames=6),
}


def _setup(name, seed=3):
    c = CASES[name]
    cfg = synth.filter_config(c["wl"], seed=seed, **c["over"])
    seq = synth.make_sequence(c["wl"], seed=1000, frames=c["frames"])
    truth = np.repeat(seq.initial_truth().astype(np.float64), cfg["n_filters"], axis=0)
    return cfg, seq.frames, truth


@pytest.mark.parametrize("name", sorted(CASES))
def test_objective_is_the_filters_own_log_z(name):
    cfg, frames, truth = _setup(name)
    J, _, tape = O.grad(cfg, truth, frames)
    o = O.Oracle(cfg, truth)
    lz = np.zeros(cfg["n_filters"])
    for k in range(frames.shape[0]):
        tr = o.step(frames[k], want={"log_z", "anc", "n_ex"})
        lz += tr["log_z"]
        assert np.array_equal(tr["anc"], tape.anc[k])
        assert np.array_equal(tr["n_ex"], tape.n_ex[k])
    assert np.array_equal(J, lz)
    # the replay with the recorded choices reproduces J exactly
    assert np.array_equal(O.replay(cfg, truth, frames, tape), J)


def _fd(cfg, truth, frames, tape, which, h):
    sig, q = float(np.float32(cfg["psf_sigma"])), float(np.float32(cfg["q"]))
    if which == 0:
        f = lambda d: O.replay(cfg, truth, frames, tape, psf_sigma=sig + d)
    elif which == 1:
        f = lambda d: O.replay(cfg, truth, frames, tape, dI0=d)
    else:
        f = lambda d: O.replay(cfg, truth, frames, tape, q=q + d)
    # Richardson-extrapolated central difference (error O(h^4))
    d1 = (f(h) - f(-h)) / (2 * h)
    d2 = (f(2 * h) - f(-2 * h)) / (4 * h)
    return (4 * d1 - d2) / 3


@pytest.mark.parametrize("name", sorted(CASES))
def test_gradient_matches_finite_differences(name):
    cfg, frames, truth = _setup(name)
    _, dJ, tape = O.grad(cfg, truth, frames)
    for j, h in enumerate((1e-4, 1e-4, 1e-4)):
        fd = _fd(cfg, truth, frames, tape, j, h)
        scale = max(1.0, np.abs(dJ[:, j]).max())
        assert np.allclose(dJ[:, j], fd, rtol=1e-6, atol=1e-6 * scale), (j, dJ[:, j], fd)


def test_gradient_terms_are_not_trivial():
    """A dropped term would not show if a derivative were zero by
    construction: every component is far from zero in every case."""
    for name in CASES:
        cfg, frames, truth = _setup(name)
        _, dJ, _ = O.grad(cfg, truth, frames)
        assert np.all(np.abs(dJ) > 1e-2), (name, dJ)


def test_single_pe_plain_sir():
    """M = 1 is plain SIR (Alg. 1, always resampling): J is the product-form
    marginal-likelihood estimate and its frozen-choice derivative still
    matches finite differences, for every component."""
    cfg, frames, truth = _setup("rna")
    cfg1 = dict(cfg, n_pe=1, n_per_pe=cfg["n_pe"] * cfg["n_per_pe"], fixed_ratio=0.0)
    _, dJ1, tape = O.grad(cfg1, truth, frames)
    assert np.all(tape.n_ex == 0)
    for j in range(3):
        fd = _fd(cfg1, truth, frames, tape, j, 1e-4)
        assert np.allclose(dJ1[:, j], fd, rtol=1e-6, atol=1e-6), (j, dJ1[:, j], fd)
