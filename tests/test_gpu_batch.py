"""Batched launches (pf_batch_*): contexts of different shapes advanced
together give bitwise the results of separate runs, with and without graph
capture, across a rebuild of the ring table."""
import numpy as np
import pytest

from paper_1310_4624_amd import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


def _cases():
    base = dict(patch=9, init_mode=0, fixed_ratio=0.1, initial_ratio=0.1, eff_cutoff=0.99,
                psf_sigma=1.5, background=5.0, noise_sigma=2.0, q=0.5, sigma_I=0.5)
    return [
        dict(base, n_filters=1, n_pe=4, n_per_pe=256, width=128, height=128, mode=0, lik_mode=0, seed=1),
        dict(base, n_filters=1, n_pe=4, n_per_pe=256, width=128, height=128, mode=1, lik_mode=0, seed=2),
        dict(base, n_filters=2, n_pe=8, n_per_pe=300, width=96, height=80, mode=1, lik_mode=0, seed=3),
        dict(base, n_filters=1, n_pe=6, n_per_pe=2500, width=128, height=128, mode=1, lik_mode=0, seed=4),
        dict(base, n_filters=1, n_pe=4, n_per_pe=1000, width=64, height=48, mode=1, lik_mode=2,
             background=10.0, seed=5),
        dict(base, n_filters=3, n_pe=5, n_per_pe=77, width=128, height=128, mode=0, lik_mode=1,
             fixed_ratio=0.5, noise_sigma=1.0, seed=6),
        dict(base, n_filters=1, n_pe=3, n_per_pe=200, width=64, height=64, mode=1, lik_mode=0,
             patch=7, seed=7),                                   # no batched variant: solo
        dict(base, n_filters=1, n_pe=5, n_per_pe=1000, width=96, height=80, mode=1, lik_mode=0,
             block_size=512, seed=8),                            # 2 slots per thread
        dict(base, n_filters=2, n_pe=8, n_per_pe=100, width=96, height=80, mode=1, lik_mode=0,
             ring_groups=4, seed=9),
        # several PEs per workgroup, and PEs beyond LDS split over workgroups
        dict(base, n_filters=1, n_pe=4, n_per_pe=256, width=128, height=128, mode=1, lik_mode=0,
             pes_per_wg=2, seed=10),
        dict(base, n_filters=2, n_pe=3, n_per_pe=130, width=96, height=80, mode=0, lik_mode=1,
             fixed_ratio=0.5, noise_sigma=1.0, pes_per_wg=3, seed=11),
        dict(base, n_filters=1, n_pe=2, n_per_pe=5000, width=96, height=96, mode=1, lik_mode=0,
             seed=12),
        dict(base, n_filters=1, n_pe=2, n_per_pe=4500, width=64, height=64, mode=1, lik_mode=2,
             background=10.0, seed=13),
        # 512 PEs or more: master records, stepped one by one inside the run
        dict(base, n_filters=1, n_pe=600, n_per_pe=16, width=96, height=80, mode=1, lik_mode=0,
             seed=14),
        dict(base, n_filters=2, n_pe=520, n_per_pe=20, width=96, height=80, mode=1, lik_mode=0,
             pes_per_wg=4, seed=15),
    ]


def _inputs(cfg, K, rng):
    F = cfg["n_filters"]
    if cfg["lik_mode"] == 1:
        truth, obs = synth.point_sequence(int(rng.integers(1 << 30)), F, K)
        return truth[0].astype(np.float32), obs
    truth = np.zeros((F, 5), np.float32)
    truth[:, 0] = rng.uniform(20, cfg["width"] - 20, F)
    truth[:, 1] = rng.uniform(20, cfg["height"] - 20, F)
    truth[:, 2:4] = rng.uniform(-0.5, 0.5, (F, 2))
    truth[:, 4] = 12.0
    frames = []
    for k in range(K):
        t = truth.astype(np.float64).copy()
        t[:, :2] += (k + 1) * t[:, 2:4]
        if cfg["lik_mode"] == 2:
            frames.append(synth.render_poisson(t, cfg["width"], cfg["height"], 1.5, 10.0, rng))
        else:
            frames.append(synth.render(t, cfg["width"], cfg["height"], 1.5, 5.0, 2.0, rng))
    return truth, np.stack(frames)


@pytest.mark.parametrize("graph", [False, True, "replay"])
def test_batch_equals_separate_runs(graph):
    import paper_1310_4624_amd as p
    rng = np.random.Generator(np.random.PCG64(2024))
    K = 70   # crosses the ring table rebuild at iteration 65
    cases = _cases()
    inputs = [_inputs(c, K, rng) for c in cases]
    print("inputs drawn", flush=True)
    frames = [torch.from_numpy(np.ascontiguousarray(fr)).cuda() for _, fr in inputs]
    print("frames on the device", flush=True)
    solo = []
    for i, (c, (truth, _), fr) in enumerate(zip(cases, inputs, frames)):
        print(f"solo case {i}: {c['n_filters']}x{c['n_pe']}x{c['n_per_pe']}", flush=True)
        t = p.Tracker(c, truth)
        t.run(fr[:40])
        t.run(fr[40:K])
        solo.append((t.debug_get("state"), t.debug_get("pe_records"), t.estimate()))
        t.close()
    trs = [p.Tracker(c, truth) for c, (truth, _) in zip(cases, inputs)]
    b = p.Batch(trs)
    print(f"batch run (graph={graph})", flush=True)
    if graph == "replay":   # runs of 10 iterations: one graph captured, replayed
        for t0 in range(0, K, 10):
            b.run([f[t0:t0 + 10] for f in frames], graph=True)
    else:
        b.run([f[:40] for f in frames], graph=graph)
        b.run([f[40:K] for f in frames], graph=graph)
    torch.cuda.synchronize()
    print("batch run done", flush=True)
    for t, (st, rec, est) in zip(trs, solo):
        assert np.array_equal(t.debug_get("state"), st)
        assert np.array_equal(t.debug_get("pe_records"), rec)
        e = t.estimate()
        assert e["step"] == K
        for key in ("x_global", "log_mass_glob", "pe_eff", "n_ex", "n_ex_next"):
            assert np.array_equal(e[key], est[key]), key
    b.close()
    for t in trs:
        t.close()


def test_batch_rejects_bad_input():
    import paper_1310_4624_amd as p
    c = _cases()[0]
    t = p.Tracker(c, np.zeros((1, 5), np.float32))
    with pytest.raises(p.PFError):
        p.Batch([t, t])                                          # the same context twice
    b = p.Batch([t])
    t.grad_begin(2)
    fr = torch.zeros((2, 128, 128), dtype=torch.float32, device="cuda")
    with pytest.raises(p.PFError):
        b.run([fr])                                              # recording a gradient
    t.grad_end(fr[:0])
    b.run([fr])
    b.close()
    t.close()


def test_autotuner_and_batched_workload():
    """The autotuner returns one of its candidates; a small instance of the
    batched workload runs in every mode with the separate runs' results."""
    from paper_1310_4624_amd import autotune
    from paper_1310_4624_amd.experiments import batch
    seqs = synth.batch_sequences(seed=7, n_seq=3, frames=8)
    c, t, fr = seqs[0]
    b = autotune.tune(c, t, torch.from_numpy(fr).cuda(), steps=4)
    assert (b["block_size"], b["pes_per_wg"]) in autotune.shapes(c["n_per_pe"], c["n_pe"])
    out = batch(frames=6, n_seq=4, seed=7)
    assert out["batched_equal"] and out["batched_graph_equal"]
    assert len(out["tuned_shapes"]) == 4
