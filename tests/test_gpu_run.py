"""Multi-iteration launches (pf_config.launch): every PE's workgroup stays
resident for up to 64 iterations, its resampled particles held in registers,
and the PEs of a filter meet at a barrier between iterations.  The arithmetic
is that of one launch per iteration, so every output must agree bitwise with
a stepwise run of the same context: particles, PE records, N_ex, estimates.
The stepwise path itself is held to the oracle by the parity tests."""
import numpy as np
import pytest

from paper_1310_4624_amd import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

STEPWISE, PERSISTENT = 1, 2


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


BASE = dict(patch=9, init_mode=0, fixed_ratio=0.1, initial_ratio=0.1, eff_cutoff=0.99,
            psf_sigma=1.5, background=5.0, noise_sigma=2.0, q=0.5, sigma_I=0.5)

CASES = {
    # the benchmark shape: 4 filters x 64 PEs x 4096, 512 x 512; 70 iterations
    # cross the ring-table rebuild at iteration 65 (two launches: 64 + 6)
    "tracking_4x64x4096": (dict(BASE, n_filters=4, n_pe=64, n_per_pe=4096, width=512, height=512,
                                mode=1, lik_mode=0, seed=11), 70),
    "infoshare_1x256x4096": (dict(BASE, n_filters=1, n_pe=256, n_per_pe=4096, width=512,
                                  height=512, mode=1, lik_mode=0, init_mode=1, seed=12), 20),
    "rna10_2x8x4096": (dict(BASE, n_filters=2, n_pe=8, n_per_pe=4096, width=128, height=128,
                            mode=0, lik_mode=0, seed=13), 30),
    "rna50_2x8x4096": (dict(BASE, n_filters=2, n_pe=8, n_per_pe=4096, width=128, height=128,
                            mode=0, lik_mode=0, fixed_ratio=0.5, seed=14), 12),
    "poisson_1x16x2048": (dict(BASE, n_filters=1, n_pe=16, n_per_pe=2048, width=128, height=128,
                               mode=1, lik_mode=2, background=10.0, seed=15), 25),
    "arna_3x5x300": (dict(BASE, n_filters=3, n_pe=5, n_per_pe=300, width=96, height=80, mode=1,
                          lik_mode=0, seed=16), 30),
    "point_3x5x77": (dict(BASE, n_filters=3, n_pe=5, n_per_pe=77, width=128, height=128, mode=0,
                          lik_mode=1, fixed_ratio=0.5, noise_sigma=1.0, seed=17), 20),
    "groups8_1x32x4096": (dict(BASE, n_filters=1, n_pe=32, n_per_pe=4096, width=256, height=256,
                               mode=1, lik_mode=0, ring_groups=8, seed=18), 20),
    "block512_1x5x1000": (dict(BASE, n_filters=1, n_pe=5, n_per_pe=1000, width=96, height=80,
                               mode=1, lik_mode=0, block_size=512, seed=19), 20),
    "one_pe_4x1x1024": (dict(BASE, n_filters=4, n_pe=1, n_per_pe=1024, width=128, height=128,
                             mode=1, lik_mode=0, seed=20), 15),
}


def _inputs(cfg, K, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    F = cfg["n_filters"]
    if cfg["lik_mode"] == 1:
        truth, obs = synth.point_sequence(int(rng.integers(1 << 30)), F, K)
        return truth[0].astype(np.float32), obs
    W, H = cfg["width"], cfg["height"]
    truth = np.zeros((F, 5), np.float32)
    truth[:, 0] = rng.uniform(24, W - 24, F)
    truth[:, 1] = rng.uniform(24, H - 24, F)
    truth[:, 2:4] = rng.uniform(-0.4, 0.4, (F, 2))
    truth[:, 4] = 10.0
    frames = []
    for k in range(K):
        t = truth.astype(np.float64).copy()
        t[:, :2] += (k + 1) * t[:, 2:4]
        if cfg["lik_mode"] == 2:
            frames.append(synth.render_poisson(t, W, H, 1.5, 10.0, rng))
        else:
            frames.append(synth.render(t, W, H, 1.5, 5.0, 2.0, rng))
    return truth, np.stack(frames).astype(np.float32)


def _outputs(t):
    e = t.estimate()
    return dict(state=t.debug_get("state"), rec=t.debug_get("pe_records"),
                **{k: e[k] for k in ("x_global", "log_mass_glob", "pe_eff", "n_ex", "n_ex_next",
                                     "log_z_inc", "step")})


def _assert_same(a, b, name):
    for k in a:
        assert np.array_equal(a[k], b[k], equal_nan=True), (name, k)


def _run(cfg, truth, frames, launch, chunks):
    import paper_1310_4624_amd as p
    t = p.Tracker(dict(cfg, launch=launch), truth)
    assert t.multi_iteration() == (launch == PERSISTENT)
    i = 0
    for n in chunks:
        if n == "step":
            t.step(frames[i])
            i += 1
        else:
            t.run(frames[i:i + n])
            i += n
    torch.cuda.synchronize()
    out = _outputs(t)
    t.close()
    return out


@pytest.mark.parametrize("name", list(CASES))
def test_multi_iteration_launch_equals_stepwise(name):
    cfg, K = CASES[name]
    print(f"case {name} K={K}", flush=True)
    truth, fr = _inputs(cfg, K, 1000 + cfg["seed"])
    frames = torch.from_numpy(np.ascontiguousarray(fr)).cuda()
    ref = _run(cfg, truth, frames, STEPWISE, [K])
    got = _run(cfg, truth, frames, PERSISTENT, [K])
    assert got["step"] == K
    _assert_same(got, ref, name)


def test_mixed_calls_and_lone_iterations():
    """pf_step, a one-iteration pf_run (a k_step launch) and multi-iteration
    runs interleaved continue one another exactly (first-iteration ratio,
    ping-pong parity, ring rows)."""
    cfg, _ = CASES["groups8_1x32x4096"]
    cfg = dict(cfg, ring_groups=0, seed=31)
    K = 75
    truth, fr = _inputs(cfg, K, 77)
    frames = torch.from_numpy(fr).cuda()
    ref = _run(cfg, truth, frames, STEPWISE, [K])
    got = _run(cfg, truth, frames, PERSISTENT, ["step", 1, 30, 1, 2, 40])
    _assert_same(got, ref, "mixed")


def test_timed_run_and_state_load():
    """pf_run_timed gives every iteration a positive time and the same results;
    a state loaded with pf_debug_set_state is picked up by the first
    iteration of a multi-iteration launch."""
    import paper_1310_4624_amd as p
    cfg, _ = CASES["rna10_2x8x4096"]
    K = 20
    truth, fr = _inputs(cfg, K, 5)
    frames = torch.from_numpy(fr).cuda()
    outs = []
    for launch in (STEPWISE, PERSISTENT):
        t = p.Tracker(dict(cfg, launch=launch), truth)
        t.run(frames[:5])
        st = t.debug_get("state")
        lm = t.debug_get("logmass")
        rng = np.random.Generator(np.random.PCG64(9))
        st = (st + rng.normal(0, 0.5, st.shape)).astype(np.float32)
        t.set_state(st, lm, step=5)
        ms = t.run_timed(frames[5:K])
        assert ms.shape == (K - 5,) and np.all(ms > 0)
        outs.append(_outputs(t))
        t.close()
    _assert_same(outs[1], outs[0], "timed")


def test_gradient_recording_runs_stepwise():
    """While a gradient tape records, iterations run one launch each; the
    value and gradient match a stepwise context's."""
    import paper_1310_4624_amd as p
    cfg, _ = CASES["rna10_2x8x4096"]
    K = 6
    truth, fr = _inputs(cfg, K, 6)
    frames = torch.from_numpy(fr).cuda()
    res = []
    for launch in (STEPWISE, PERSISTENT):
        t = p.Tracker(dict(cfg, launch=launch), truth)
        t.grad_begin(K)
        t.run(frames)
        g = t.grad_end(frames)
        res.append(g)
        t.close()
    for k in res[0]:
        assert np.array_equal(np.asarray(res[0][k]), np.asarray(res[1][k])), k


def test_contexts_that_cannot_stay_resident_are_refused():
    import paper_1310_4624_amd as p
    z = np.zeros((1, 5), np.float32)
    bad = [
        dict(BASE, n_filters=2, n_pe=256, n_per_pe=4096, width=512, height=512, mode=1,
             lik_mode=0, seed=1),                     # 512 workgroups of 127 KiB LDS
        dict(BASE, n_filters=1, n_pe=4, n_per_pe=256, width=128, height=128, mode=1,
             lik_mode=0, patch=7, seed=1),            # no multi-iteration variant
    ]
    for c in bad:
        with pytest.raises(p.PFError) as e:
            p.Tracker(dict(c, launch=PERSISTENT), np.zeros((c["n_filters"], 5), np.float32))
        assert e.value.code == -6                     # PF_EUNSUPPORTED
        t = p.Tracker(dict(c, launch=0), np.zeros((c["n_filters"], 5), np.float32))
        assert not t.multi_iteration()                # AUTO falls back to stepwise
        t.close()
    c = dict(BASE, n_filters=1, n_pe=4, n_per_pe=256, width=128, height=128, mode=1, lik_mode=0,
             seed=1)
    with pytest.raises(p.PFError):
        p.Tracker(dict(c, launch=PERSISTENT), z, debug=1)   # trace buffers: stepwise only
    t = p.Tracker(dict(c, launch=PERSISTENT), z)
    assert t.multi_iteration()
    t.close()
    # AUTO: one launch per iteration, whatever the size
    for F, M, want in ((1, 4, False), (4, 16, False), (1, 65, False), (4, 64, False)):
        c = dict(BASE, n_filters=F, n_pe=M, n_per_pe=1024, width=128, height=128, mode=1,
                 lik_mode=0, seed=1)
        t = p.Tracker(dict(c, launch=0), np.zeros((F, 5), np.float32))
        assert t.multi_iteration() == want, (F, M)
        t.close()
