"""The reverse sweep of the GPU path against the oracle's forward-mode
gradient (itself pinned to finite differences in test_oracle_grad.py).

Both sides run the same iterations from the same start with the same seed;
the comparison needs the same discrete choices, which is checked first: the
GPU's ancestors and N_ex of every iteration equal the oracle's (the integer
stage is bit-exact; a quantization tie could flip an ancestor, and these
seeds have none).  Then J and dJ/dtheta, theta = (psf_sigma, I0, q), are
compared to 1e-3 relative.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1310_4624_amd import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


def pf():
    import paper_1310_4624_amd as p
    return p


CASES = {
    "rna_4x256": dict(over={}, frames=8),
    "arna_2x8x128": dict(over=dict(mode=O.MODE_ARNA, n_filters=2, n_pe=8, n_per_pe=128), frames=8),
    "arna_infoshare_6x256": dict(over=dict(mode=O.MODE_ARNA, init_mode=O.INIT_INFOSHARE, n_pe=6,
                                           n_per_pe=256), frames=6),
    "arna_2x4096": dict(over=dict(mode=O.MODE_ARNA, n_pe=2, n_per_pe=4096), frames=5),
    "rna_border_3x1000": dict(over=dict(n_pe=3, n_per_pe=1000, width=40, height=40), frames=6),
    # forward iterations with several PEs per workgroup (the adjoint is the same)
    "grouped_arna_2x8x128": dict(over=dict(mode=O.MODE_ARNA, n_filters=2, n_pe=8, n_per_pe=128,
                                           pes_per_wg=4), frames=8),
    # 512 PEs or more: the forward steps take the master step from k_master,
    # the reverse sweep recomputes it from the records
    "master_arna_600x64": dict(over=dict(mode=O.MODE_ARNA, n_pe=600, n_per_pe=64), frames=6),
    "master_grouped_arna_600x64": dict(over=dict(mode=O.MODE_ARNA, n_pe=600, n_per_pe=64,
                                                 pes_per_wg=4), frames=6),
    # the differentiable workload's shape: 2^20 particles over 256 PEs, 512 x 512
    "c5_arna_256x4096": dict(workload="arna_grad_512_256x4096", over={}, frames=12),
}


def _setup(name, seed=3):
    c = CASES[name]
    wl = c.get("workload", "rna_128_4x256")
    cfg = synth.filter_config(wl, seed=seed, **c["over"])
    K = c["frames"]
    if "width" in c["over"]:
        # a spot starting next to the corner of a small frame: patches cross
        # the image border
        rng = np.random.Generator(np.random.PCG64(7))
        tr = np.zeros((K + 1, 1, 5))
        for k in range(K + 1):
            tr[k, 0] = [2.5 + 0.6 * k, 3.2 + 0.4 * k, 0.6, 0.4, 20.0]
        frames = np.stack([synth.render(tr[k], cfg["width"], cfg["height"], cfg["psf_sigma"],
                                        cfg["background"], cfg["noise_sigma"], rng)
                           for k in range(1, K + 1)])
        truth0 = tr[0].astype(np.float32)
    else:
        seq = synth.make_sequence(wl, seed=1000, frames=K)
        frames, truth0 = seq.frames, seq.initial_truth()
    truth = np.repeat(truth0, cfg["n_filters"], axis=0)
    return cfg, frames, truth


def _gpu_run(cfg, truth, frames, tape=None):
    """K iterations on the GPU with recording, then the reverse sweep.  With
    `tape`, every iteration replays the oracle's ancestors and N_ex (the GPU
    path's own choices differ from the FP64 ones at quantization ties, after
    which the two runs are different runs)."""
    p = pf()
    K = frames.shape[0]
    fr = torch.from_numpy(frames).cuda()
    tr = p.Tracker(cfg, truth)
    tr.grad_begin(K)
    if tape is None:
        tr.run(fr)
    else:
        for k in range(K):
            tr.force_next(anc=tape.anc[k], nex=tape.n_ex[k])
            tr.step(fr[k])
    Jv = tr.grad_value()
    res = tr.grad_end(fr)
    tr.close()
    return Jv, res


@pytest.mark.parametrize("name", sorted(CASES))
def test_gradient_matches_oracle(name):
    print(f"case {name}", flush=True)
    cfg, frames, truth = _setup(name)
    J, dJ, tape = O.grad(cfg, truth.astype(np.float64), frames)
    Jv, res = _gpu_run(cfg, truth, frames, tape=tape)
    assert np.allclose(res["J"], J, rtol=1e-5, atol=1e-3), (res["J"], J)
    assert np.array_equal(Jv, res["J"])
    assert np.allclose(res["grad"], dJ, rtol=1e-3, atol=1e-4 * np.abs(dJ).max()), (res["grad"], dJ)


def test_free_run_choices_mostly_agree():
    """Without replay the GPU makes the same choices as the oracle except at
    rare quantization ties (checked on the first iteration, before any tie
    can change the states)."""
    p = pf()
    # (the small shapes: at 2^20 particles the one-step parity test compares
    # every ancestor against the oracle with the quantization tolerance)
    for name in sorted(n for n in CASES if "workload" not in CASES[n]):
        cfg, frames, truth = _setup(name)
        _, _, tape = O.grad(cfg, truth.astype(np.float64), frames[:1])
        tr = p.Tracker(cfg, truth, debug=p.PF_DEBUG_TRACE)
        tr.step(torch.from_numpy(frames[:1]).cuda()[0])
        anc = tr.debug_get("ancestors")
        assert np.array_equal(tr.estimate()["n_ex"], tape.n_ex[0])
        tr.close()
        assert np.count_nonzero(anc != tape.anc[0]) <= max(2, anc.size // 500), name


def test_gradient_deterministic_and_state_continues():
    """Two recordings give bit-identical results, and recording changes
    nothing in the filter: the state after grad_end equals that of a run
    without recording, and later iterations continue identically."""
    p = pf()
    cfg, frames, truth = _setup("arna_2x8x128")
    fr = torch.from_numpy(frames).cuda()
    outs, states = [], []
    for rec in (True, True, False):
        tr = p.Tracker(cfg, truth)
        if rec:
            tr.grad_begin(5)
        tr.run(fr[:5])
        if rec:
            outs.append(tr.grad_end(fr[:5]))
        tr.run(fr[5:])
        states.append((tr.debug_get("state"), tr.estimate()["x_global"]))
        tr.close()
    assert np.array_equal(outs[0]["grad"], outs[1]["grad"])
    assert np.array_equal(outs[0]["J"], outs[1]["J"])
    for s in states[1:]:
        assert np.array_equal(s[0], states[0][0])
        assert np.array_equal(s[1], states[0][1])


def test_recording_limits():
    p = pf()
    cfg, frames, truth = _setup("rna_4x256")
    fr = torch.from_numpy(frames).cuda()
    tr = p.Tracker(cfg, truth)
    with pytest.raises(p.PFError):
        tr.grad_end(fr)                       # not recording
    tr.grad_begin(2)
    with pytest.raises(p.PFError):
        tr.grad_begin(2)                      # already recording
    tr.run(fr[:2])
    with pytest.raises(p.PFError):
        tr.step(fr[2])                        # tape full
    out = tr.grad_end(fr[:2])
    assert np.all(np.isfinite(out["grad"]))
    tr.step(fr[2])                            # recording over: steps run again
    tr.grad_begin(1)
    assert np.array_equal(tr.grad_end(fr[:0])["grad"], np.zeros((1, 3)))   # nothing recorded
    tr.close()
    pc = dict(cfg, lik_mode=p.PF_LIK_POINT)
    tp = p.Tracker(pc, truth)
    with pytest.raises(p.PFError):
        tp.grad_begin(1)
    tp.close()


def test_autograd_function():
    """torch.autograd drives the same sweep: J and theta.grad equal the
    summed results of the same run through the Tracker."""
    from paper_1310_4624_amd.grad import log_marginal
    p = pf()
    cfg, frames, truth = _setup("arna_2x8x128")
    fr = torch.from_numpy(frames).cuda()
    th0 = np.array([np.float32(cfg["psf_sigma"]), truth[0, 4], np.float32(cfg["q"])], np.float64)
    theta = torch.tensor(th0, dtype=torch.float64, requires_grad=True)
    J = log_marginal(theta, fr, cfg, truth)
    J.sum().backward()
    tr = p.Tracker(cfg, truth)
    tr.grad_begin(frames.shape[0])
    tr.run(fr)
    ref = tr.grad_end(fr)
    tr.close()
    assert np.array_equal(J.detach().cpu().numpy(), ref["J"])
    assert np.array_equal(theta.grad.numpy(), ref["grad"].sum(0))
