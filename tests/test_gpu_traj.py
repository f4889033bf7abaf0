"""Per-iteration master steps on the device (pf_run_traj): row i of the
trajectory is the master step of iteration i (Alg. 3, steps 9-10) -- the
same bits pf_estimate reports after that iteration of a stepwise run -- and
it agrees with the oracle's master step computed from the device's own PE
records."""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_1310_4624_amd import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


BASE = dict(patch=9, init_mode=0, fixed_ratio=0.1, initial_ratio=0.1, eff_cutoff=0.99,
            psf_sigma=1.5, background=5.0, noise_sigma=2.0, q=0.5, sigma_I=0.5)

CASES = {
    "arna_2x8x1024": dict(BASE, n_filters=2, n_pe=8, n_per_pe=1024, width=128, height=128,
                          mode=1, lik_mode=0, seed=41),
    "rna_1x16x300": dict(BASE, n_filters=1, n_pe=16, n_per_pe=300, width=96, height=80,
                         mode=0, lik_mode=0, seed=42),
    "point_3x5x77": dict(BASE, n_filters=3, n_pe=5, n_per_pe=77, width=128, height=128, mode=1,
                         lik_mode=1, noise_sigma=1.0, seed=43),
    "persistent_1x4x256": dict(BASE, n_filters=1, n_pe=4, n_per_pe=256, width=128, height=128,
                               mode=1, lik_mode=0, launch=2, seed=44),
    # several PEs per workgroup; PEs split over workgroups (rows from k_global)
    "grouped_2x8x200": dict(BASE, n_filters=2, n_pe=8, n_per_pe=200, width=128, height=128,
                            mode=1, lik_mode=0, pes_per_wg=4, seed=45),
    "split_1x4x9000": dict(BASE, n_filters=1, n_pe=4, n_per_pe=9000, width=128, height=128,
                           mode=1, lik_mode=0, seed=46),
    # 512 PEs or more: the master step once per filter after every step
    # (k_master, from the records after k_step, from the log-masses k_step_flex
    # writes beside them), rows from k_global
    "master_1x600x64": dict(BASE, n_filters=1, n_pe=600, n_per_pe=64, width=128, height=128,
                            mode=1, lik_mode=0, seed=47),
    "master_grouped_2x1100x50": dict(BASE, n_filters=2, n_pe=1100, n_per_pe=50, width=128,
                                     height=128, mode=1, lik_mode=0, pes_per_wg=4, seed=48),
}
KEYS = ("x_global", "log_mass_glob", "pe_eff", "n_ex", "n_ex_next", "log_z_inc")


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
        frames.append(synth.render(t, W, H, 1.5, 5.0, 2.0, rng))
    return truth, np.stack(frames).astype(np.float32)


@pytest.mark.parametrize("name", list(CASES))
def test_trajectory_rows_are_the_stepwise_estimates(name):
    import paper_1310_4624_amd as p
    cfg = CASES[name]
    K, F = 12, cfg["n_filters"]
    print(f"case {name} K={K}", flush=True)
    truth, fr = _inputs(cfg, K, 500 + cfg["seed"])
    frames = torch.from_numpy(np.ascontiguousarray(fr)).cuda()
    a = p.Tracker(cfg, truth)
    traj = torch.zeros(K * F * p.TRAJ_RECORD_BYTES, dtype=torch.uint8, device="cuda")
    a.run_traj(frames[:5], traj[:5 * F * p.TRAJ_RECORD_BYTES])
    a.run_traj(frames[5:], traj[5 * F * p.TRAJ_RECORD_BYTES:])
    torch.cuda.synchronize()
    tr = p.trajectory(traj, K, F)
    b = p.Tracker(cfg, truth)
    for k in range(K):
        b.step(frames[k])
        e = b.estimate()
        assert np.array_equal(tr["step"][k], np.full(F, k + 1))
        got = dict(x_global=tr["xhat"][k].reshape(-1), log_mass_glob=tr["log_mass_glob"][k],
                   pe_eff=tr["pe_eff"][k], n_ex=tr["n_ex"][k], n_ex_next=tr["n_ex_next"][k],
                   log_z_inc=tr["log_z_inc"][k])
        for key in KEYS:
            assert np.array_equal(got[key], np.asarray(e[key]).reshape(-1), equal_nan=True), (k, key)
    # the context continues as a plain run would
    assert np.array_equal(a.debug_get("state"), b.debug_get("state"))
    # the last row against the oracle's master step of the device's records
    rec = b.debug_get("pe_records")   # [F][M]: log W^(m), x^m (5), lstar, T
    for f in range(F):
        ref = orc.master(cfg, rec[f, :, 0], rec[f, :, 1:6])
        assert tr["n_ex_next"][K - 1][f] == ref["n_ex_next"]
        assert np.isclose(tr["log_mass_glob"][K - 1][f], ref["L_glob"], rtol=0, atol=1e-10)
        assert np.isclose(tr["pe_eff"][K - 1][f], ref["pe_eff"], rtol=1e-12, atol=0)
        assert np.isclose(tr["log_z_inc"][K - 1][f], ref["log_z"], rtol=0, atol=1e-10)
        assert np.allclose(tr["xhat"][K - 1][f], ref["xhat"], rtol=1e-12, atol=1e-9)
    a.close()
    b.close()


def test_trajectory_rejects_misaligned_buffer():
    import paper_1310_4624_amd as p
    cfg = CASES["rna_1x16x300"]
    truth, fr = _inputs(cfg, 2, 7)
    frames = torch.from_numpy(np.ascontiguousarray(fr)).cuda()
    t = p.Tracker(cfg, truth)
    buf = torch.zeros(2 * p.TRAJ_RECORD_BYTES + 8, dtype=torch.uint8, device="cuda")
    with pytest.raises(p.PFError):
        t.run_traj(frames, buf[1:])
    t.close()
