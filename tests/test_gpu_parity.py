"""GPU path (through the C interface) against the FP64 oracle.

Integer stages are compared bit for bit on identical integer inputs; the float
stages of one iteration are compared element by element from identical float32
starting states, within the tolerances derived in tests/helpers.py; multi-step
runs are compared on what is unique (N_ex, rings) and statistically.
"""
import ctypes
import zlib

import numpy as np
import pytest

import oracle.oracle as orc
from paper_1310_4624_amd import synth
from tests import helpers as H

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    import paper_1310_4624_amd  # noqa: F401


def pf():
    import paper_1310_4624_amd as p
    return p


SEED = 0x51D_2013


# ------------------------------------------------------------- integer stages
def test_device_philox_bit_exact():
    p = pf()
    rng = np.random.Generator(np.random.PCG64(1))
    ctr = rng.integers(0, 2 ** 32, (4096, 4), dtype=np.uint64).astype(np.uint32)
    key = np.array([0xDEADBEEF, 0x01234567], np.uint32)
    got = p.philox(ctr, key)
    for i in range(0, 4096, 97):
        assert np.array_equal(got[i], orc.philox(ctr[i], key))
    kat = np.array([[0, 0, 0, 0], [0xFFFFFFFF] * 4], np.uint32)
    assert list(p.philox(kat[:1], [0, 0])[0]) == [0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8]
    assert list(p.philox(kat[1:], [0xFFFFFFFF, 0xFFFFFFFF])[0]) == [0x408F276D, 0x41C83B0E,
                                                                    0xA20BC7C6, 0x6D5451FD]


@pytest.mark.parametrize("n_p", [1, 2, 3, 63, 64, 65, 100, 256, 1000, 1024, 1025, 2048, 3333, 4096])
def test_device_resampling_bit_exact(n_p):
    p = pf()
    rng = np.random.Generator(np.random.PCG64(n_p))
    qm = orc.qmax(n_p)
    blocks = []
    for b in range(6):
        kind = ["mixed", "uniform", "spike", "mixed", "mixed", "mixed"][b]
        blocks.append(synth.random_weights_q(rng, n_p, qm, kind))
    Q = np.stack(blocks)
    T = Q.astype(np.int64).sum(axis=1)
    V = np.array([rng.integers(0, t) for t in T], np.uint32)
    V[0] = 0
    V[1] = T[1] - 1
    got = p.resample_q(Q, V)
    for b in range(len(blocks)):
        assert np.array_equal(got[b], orc.resample(Q[b], int(V[b]))), b


def test_device_exchange_count_bit_exact():
    p = pf()
    rng = np.random.Generator(np.random.PCG64(2))
    for trial in range(200):
        M = int(rng.integers(1, 8193 if trial % 20 == 0 else 400))
        n_p = int(rng.integers(1, 65537 if trial % 4 == 0 else 4097))
        P = np.floor(np.exp(-rng.exponential(rng.uniform(0.05, 8), M)) * 2 ** 20).astype(np.uint32)
        P[rng.integers(0, M)] = 1 << 20
        for mode, first in [(1, False), (1, True), (0, False)]:
            cut = float(rng.choice([0.99, 0.5, 1.0, 0.0]))
            a = p.nex(P, n_p, mode=mode, fixed_ratio=0.3, initial_ratio=0.1, cutoff=cut,
                      first=first)
            b = orc.nex(P, n_p, mode=mode, fixed_ratio=0.3, initial_ratio=0.1, cutoff=cut,
                        first=first)
            assert a == b, (M, n_p, mode, first, cut)
    P = np.full(100, 1 << 20, np.uint32)
    P[99] = 0
    assert p.nex(P, 4096) == orc.nex(P, 4096) == 4096 // 198
    P[99] = 1
    assert p.nex(P, 4096) == 0


@pytest.mark.parametrize("M", [1, 2, 3, 5, 64, 256, 257, 1000])
def test_device_ring_bit_exact(M):
    p = pf()
    for f in [0, 3]:
        for k in [1, 2, 63, 64, 65, 1000]:
            got = p.ring(SEED, f, k, M)
            _, want, _ = orc.ring(SEED, f, k, M)
            assert np.array_equal(got, want), (M, f, k)
    assert np.array_equal(p.ring(SEED, 0, 5, M, mode=0), (np.arange(M) - 1) % M)


@pytest.mark.parametrize("M,G", [(2, 8), (7, 8), (8, 8), (64, 8), (256, 8), (1000, 8), (300, 3),
                                 (4096, 256), (100, 100), (8192, 7)])
def test_device_grouped_ring_bit_exact(M, G):
    p = pf()
    for f in [0, 1, 5]:
        for k in [1, 64, 777]:
            got = p.ring(SEED, f, k, M, groups=G)
            _, want, _ = orc.ring_groups(SEED, f, k, M, G)
            assert np.array_equal(got, want), (M, G, f, k)


# ------------------------------------------------------- one-step float parity
def seeded_case(name):
    rng = np.random.Generator(np.random.PCG64(zlib.crc32(name.encode())))
    if name == "rna_128_4x256":
        seq = synth.make_sequence("rna_128_4x256", seed=1003, frames=6)
        cfg = synth.filter_config("rna_128_4x256", seed=SEED)
        frame = seq.frames[5]
        centre = seq.truth[5, :1, :2]
    elif name == "arna_ragged_2x3x100":
        cfg = dict(n_filters=2, n_pe=3, n_per_pe=100, width=96, height=80, patch=9,
                   mode=1, init_mode=0, lik_mode=0, fixed_ratio=0.1, initial_ratio=0.1,
                   eff_cutoff=0.99, psf_sigma=1.5, background=5.0, noise_sigma=2.0, q=0.5,
                   sigma_I=0.5, seed=SEED + 1)
        truth = np.array([[[30.3, 40.7, 0, 0, 12.0], [70.6, 20.2, 0, 0, 9.0]]])
        frame = synth.render(truth[0], 96, 80, 1.5, 5.0, 2.0, rng)
        centre = truth[0, :, :2]
    elif name == "arna_1x6x2500":
        cfg = dict(n_filters=1, n_pe=6, n_per_pe=2500, width=128, height=128, patch=9,
                   mode=1, init_mode=0, lik_mode=0, fixed_ratio=0.1, initial_ratio=0.1,
                   eff_cutoff=0.99, psf_sigma=1.5, background=5.0, noise_sigma=2.0, q=0.5,
                   sigma_I=0.5, seed=SEED + 2)
        truth = np.array([[[64.2, 63.9, 0, 0, 8.0]]])
        frame = synth.render(truth[0], 128, 128, 1.5, 5.0, 2.0, rng)
        centre = truth[0, :, :2]
    elif name == "arna_groups_2x24x300":
        # hardware-aware ring: 8 groups
        cfg = dict(n_filters=2, n_pe=24, n_per_pe=300, width=96, height=80, patch=9,
                   mode=1, init_mode=0, lik_mode=0, fixed_ratio=0.1, initial_ratio=0.1,
                   eff_cutoff=0.99, psf_sigma=1.5, background=5.0, noise_sigma=2.0, q=0.5,
                   sigma_I=0.5, seed=SEED + 6, ring_groups=8)
        truth = np.array([[[30.3, 40.7, 0, 0, 12.0], [70.6, 20.2, 0, 0, 9.0]]])
        frame = synth.render(truth[0], 96, 80, 1.5, 5.0, 2.0, rng)
        centre = truth[0, :, :2]
    elif name == "poisson_arna_1x4x1000":
        cfg = dict(n_filters=1, n_pe=4, n_per_pe=1000, width=64, height=48, patch=9,
                   mode=1, init_mode=0, lik_mode=2, fixed_ratio=0.1, initial_ratio=0.1,
                   eff_cutoff=0.99, psf_sigma=1.5, background=10.0, noise_sigma=1.0, q=0.5,
                   sigma_I=0.5, seed=SEED + 4)
        truth = np.array([[[20.4, 30.6, 0, 0, 20.0], [58.2, 3.1, 0, 0, 15.0]]])
        frame = synth.render_poisson(truth[0], 64, 48, 1.5, 10.0, rng)
        centre = truth[0, :1, :2]
    elif name == "arna_2x2100x4":
        # many small PEs: the master step is computed once per filter
        cfg = dict(n_filters=2, n_pe=2100, n_per_pe=4, width=96, height=80, patch=9,
                   mode=1, init_mode=0, lik_mode=0, fixed_ratio=0.1, initial_ratio=0.1,
                   eff_cutoff=0.99, psf_sigma=1.5, background=5.0, noise_sigma=2.0, q=0.5,
                   sigma_I=0.5, seed=SEED + 5)
        truth = np.array([[[30.3, 40.7, 0, 0, 12.0], [70.6, 20.2, 0, 0, 9.0]]])
        frame = synth.render(truth[0], 96, 80, 1.5, 5.0, 2.0, rng)
        centre = truth[0, :, :2]
    elif name in ("full_tracking_4x64x4096", "full_infoshare_256x4096",
                  "full_tracking_64x64x4096"):
        # the two 2^20 workloads in the launch configuration bench.py times
        # (and the tracking workload at 2^24); the information-sharing case
        # with spread PEs (most patches read the frame, not the tile)
        wl = {"full_tracking_4x64x4096": "arna_tracking_512_4x64x4096",
              "full_infoshare_256x4096": "arna_infoshare_512_256x4096",
              "full_tracking_64x64x4096": "arna_tracking_512_64x64x4096"}[name]
        cfg = synth.filter_config(wl, seed=SEED + 7)
        seq = synth.make_sequence(wl, seed=1004, frames=3)
        frame = seq.frames[2]
        centre = seq.truth[3, :, :2]
        F, M, n_p = cfg["n_filters"], cfg["n_pe"], cfg["n_per_pe"]
        spread = 1.5 if name.startswith("full_tracking") else 40.0
        state = synth.random_state(rng, F, M, n_p, cfg["width"], cfg["height"], spread=spread,
                                   centre=centre, I0=10.0)
        return cfg, np.asarray(frame, np.float32), state, rng.normal(0.0, 3.0, (F, M))
    elif name in ("arna_1x256x4100", "arna_1x512x4100"):
        # streamed PEs: one workgroup per PE (no split), every PE compared;
        # at 512 PEs the master step is computed once per filter
        M = 256 if name == "arna_1x256x4100" else 512
        cfg = dict(n_filters=1, n_pe=M, n_per_pe=4100, width=256, height=256, patch=9,
                   mode=1, init_mode=0, lik_mode=0, fixed_ratio=0.1, initial_ratio=0.1,
                   eff_cutoff=0.99, psf_sigma=1.5, background=5.0, noise_sigma=2.0, q=0.5,
                   sigma_I=0.5, seed=SEED + (14 if M == 256 else 15))
        truth = np.array([[[100.3, 120.6, 0, 0, 12.0]]])
        frame = synth.render(truth[0], 256, 256, 1.5, 5.0, 2.0, rng)
        state = synth.random_state(rng, 1, M, 4100, 256, 256, spread=3.0,
                                   centre=truth[0, :, :2], I0=10.0)
        return cfg, np.asarray(frame, np.float32), state, rng.normal(0.0, 3.0, (1, M))
    elif name in ("arna_2x4x16384", "arna_1x3x65536"):
        # PEs beyond the LDS stage (the streaming step): 2 spots on 256^2
        # around which the particles sit, and 1 spot on 512^2 with the
        # particles spread wider (patches from the tile and from the frame)
        F, M, n_p, side, spread = ((2, 4, 16384, 256, 1.5) if name == "arna_2x4x16384"
                                   else (1, 3, 65536, 512, 6.0))
        cfg = dict(n_filters=F, n_pe=M, n_per_pe=n_p, width=side, height=side, patch=9,
                   mode=1, init_mode=0, lik_mode=0, fixed_ratio=0.1, initial_ratio=0.1,
                   eff_cutoff=0.99, psf_sigma=1.5, background=5.0, noise_sigma=2.0, q=0.5,
                   sigma_I=0.5, seed=SEED + 8 + F)
        truth = np.array([[[0.3 * side + 0.4, 0.6 * side + 0.7, 0, 0, 12.0],
                           [0.7 * side + 0.1, 0.3 * side + 0.2, 0, 0, 9.0]][:F]])
        frame = synth.render(truth[0], side, side, 1.5, 5.0, 2.0, rng)
        state = synth.random_state(rng, F, M, n_p, side, side, spread=spread,
                                   centre=truth[0, :, :2], I0=10.0)
        return cfg, np.asarray(frame, np.float32), state, rng.normal(0.0, 3.0, (F, M))
    elif name == "full_scaling_8192x128":
        # the strong-scaling end point at 2^20: 8192 PEs of 128 particles, one
        # spot, particles around it (the launch the scaling experiment times
        # with several PEs per workgroup)
        cfg = synth.filter_config("arna_grad_512_256x4096", seed=SEED + 13, n_pe=8192,
                                  n_per_pe=128)
        seq = synth.make_sequence("arna_grad_512_256x4096", seed=1004, frames=3)
        frame = seq.frames[2]
        state = synth.random_state(rng, 1, 8192, 128, cfg["width"], cfg["height"], spread=1.5,
                                   centre=seq.truth[3, :1, :2], I0=10.0)
        return cfg, np.asarray(frame, np.float32), state, rng.normal(0.0, 3.0, (1, 8192))
    elif name == "poisson_rna_1x2x20000":
        # ragged streaming PEs (20000 = 312 x 64 + 32) exchanging half their slots
        cfg = dict(n_filters=1, n_pe=2, n_per_pe=20000, width=128, height=96, patch=9,
                   mode=0, init_mode=0, lik_mode=2, fixed_ratio=0.5, initial_ratio=0.1,
                   eff_cutoff=0.99, psf_sigma=1.5, background=10.0, noise_sigma=1.0, q=0.5,
                   sigma_I=0.5, seed=SEED + 11)
        truth = np.array([[[40.4, 50.6, 0, 0, 20.0]]])
        frame = synth.render_poisson(truth[0], 128, 96, 1.5, 10.0, rng)
        centre = truth[0, :, :2]
    elif name == "point_arna_2x3x5000":
        cfg = dict(n_filters=2, n_pe=3, n_per_pe=5000, width=128, height=128, patch=9,
                   mode=1, init_mode=0, lik_mode=1, fixed_ratio=0.1, initial_ratio=0.1,
                   eff_cutoff=0.99, psf_sigma=1.5, background=5.0, noise_sigma=1.0, q=0.5,
                   sigma_I=0.5, seed=SEED + 12)
        centre = rng.uniform(20, 100, (2, 2))
        frame = (centre + rng.standard_normal((2, 2))).astype(np.float32)
    elif name == "point_rna_3x5x77":
        cfg = dict(n_filters=3, n_pe=5, n_per_pe=77, width=128, height=128, patch=9,
                   mode=0, init_mode=0, lik_mode=1, fixed_ratio=0.5, initial_ratio=0.1,
                   eff_cutoff=0.99, psf_sigma=1.5, background=5.0, noise_sigma=1.0, q=0.5,
                   sigma_I=0.5, seed=SEED + 3)
        centre = rng.uniform(20, 100, (3, 2))
        frame = (centre + rng.standard_normal((3, 2))).astype(np.float32)
    else:
        raise KeyError(name)
    F, M, n_p = cfg["n_filters"], cfg["n_pe"], cfg["n_per_pe"]
    state = synth.random_state(rng, F, M, n_p, cfg["width"], cfg["height"], spread=1.5,
                               centre=centre, I0=10.0)
    logmass = rng.normal(0.0, 3.0, (F, M))
    return cfg, np.asarray(frame, np.float32), state, logmass


def gpu_outputs(g):
    out = {k: g.debug_get(k) for k in ["ring", "nex", "src", "lam", "prop", "ell", "q",
                                       "ancestors", "v", "state", "pe_records"]}
    out["est"] = g.estimate()
    return out


def oracle_step(cfg, frame, state, logmass, k_done):
    o = orc.Oracle(cfg, np.zeros((cfg["n_filters"], 5), np.float32))
    o.set_state(state.astype(np.float64), logmass, k_done)
    o.set_ambiguity(H.AMB_EPS_REL, H.AMB_EPS_ABS)
    return o.step(frame)


def run_one_step(cfg, frame, state, logmass, k_done):
    p = pf()
    F = cfg["n_filters"]
    g = p.Tracker(cfg, np.zeros((F, 5), np.float32), debug=p.PF_DEBUG_TRACE)
    g.set_state(state, logmass, step=k_done)
    g.step(torch.from_numpy(frame).cuda())
    out = gpu_outputs(g)
    g.close()
    return out, oracle_step(cfg, frame, state, logmass, k_done)


@pytest.mark.parametrize("name", ["rna_128_4x256", "arna_ragged_2x3x100", "arna_1x6x2500",
                                  "poisson_arna_1x4x1000", "arna_2x2100x4", "arna_groups_2x24x300",
                                  "point_rna_3x5x77", "full_tracking_4x64x4096",
                                  "full_infoshare_256x4096"])
@pytest.mark.parametrize("k_done", [0, 7])
def test_one_step_parity(name, k_done):
    check_one_step(name, k_done)


@pytest.mark.parametrize("name", ["arna_2x4x16384", "arna_1x3x65536", "poisson_rna_1x2x20000",
                                  "point_arna_2x3x5000", "arna_1x256x4100", "arna_1x512x4100"])
@pytest.mark.parametrize("k_done", [0, 7])
def test_one_step_parity_streaming(name, k_done):
    """PEs of more than 4096 particles, every PE: split over several
    workgroups (fewer than 256 PEs), else one streamed PE per workgroup."""
    check_one_step(name, k_done)


def test_one_step_parity_2e24():
    """The tracking workload at 2^24 particles (64 filters x 64 PEs x 4096,
    4096 workgroups), one step after seven."""
    check_one_step("full_tracking_64x64x4096", 7)


@pytest.mark.parametrize("name,ppw", [("rna_128_4x256", 4), ("arna_ragged_2x3x100", 2),
                                      ("arna_2x2100x4", 16), ("poisson_arna_1x4x1000", 4),
                                      ("point_rna_3x5x77", 3), ("arna_groups_2x24x300", 8),
                                      ("full_scaling_8192x128", 16)])
@pytest.mark.parametrize("k_done", [0, 7])
def test_one_step_parity_grouped(name, ppw, k_done):
    """Several PEs per workgroup (pes_per_wg), every PE."""
    check_one_step(name, k_done, pes_per_wg=ppw)


def check_one_step(name, k_done, **over):
    print(f"one-step parity {name} k_done={k_done} {over}", flush=True)
    cfg, frame, state, logmass = seeded_case(name)
    cfg = dict(cfg, **over)
    g, tr = run_one_step(cfg, frame, state, logmass, k_done)
    compare_one_step(cfg, frame, g, tr, k_done)


BATCH_CASES = ["rna_128_4x256", "arna_ragged_2x3x100", "arna_1x6x2500", "poisson_arna_1x4x1000",
               "point_rna_3x5x77", "arna_groups_2x24x300", "point_arna_2x3x5000"]


def test_one_step_parity_batched():
    """One iteration of a mixed batch (pf_batch_run: contexts of different
    shapes, likelihoods and kernel variants in shared launches) against the
    oracle, context by context, with the bar of the single-context test."""
    p = pf()
    k_done = 3
    cases = [seeded_case(n) for n in BATCH_CASES]
    trs = []
    for cfg, frame, state, logmass in cases:
        g = p.Tracker(cfg, np.zeros((cfg["n_filters"], 5), np.float32), debug=p.PF_DEBUG_TRACE)
        g.set_state(state, logmass, step=k_done)
        trs.append(g)
    b = p.Batch(trs)
    b.run([torch.from_numpy(frame[None]).cuda() for _, frame, _, _ in cases])
    torch.cuda.synchronize()
    for name, (cfg, frame, state, logmass), g in zip(BATCH_CASES, cases, trs):
        print(f"batched one-step parity {name}", flush=True)
        compare_one_step(cfg, frame, gpu_outputs(g), oracle_step(cfg, frame, state, logmass, k_done),
                         k_done)
    b.close()
    for g in trs:
        g.close()


def compare_one_step(cfg, frame, g, tr, k_done):
    F, M, n_p = cfg["n_filters"], cfg["n_pe"], cfg["n_per_pe"]
    N = F * M * n_p
    # integer stages of steps 1-3: exact
    assert np.array_equal(g["ring"], tr["ring_pred"])
    assert np.array_equal(g["nex"], tr["n_ex"])
    assert np.array_equal(g["src"], tr["src_map"])
    assert np.allclose(g["lam"], tr["lambda"], rtol=1e-6, atol=1e-6)
    # propagated particles
    tol = np.stack([H.coord_tol(tr["prop"][0]), H.coord_tol(tr["prop"][1]),
                    H.coord_tol(tr["prop"][2], 2e-5), H.coord_tol(tr["prop"][3], 2e-5),
                    H.coord_tol(tr["prop"][4])])
    assert np.all(np.abs(g["prop"] - tr["prop"]) <= tol)
    # log-likelihoods, every particle: a particle next to a pixel boundary is
    # compared with the oracle's likelihood at the patch centre the GPU took
    # (either is a valid nearest-pixel decision); the oracle then redoes
    # steps 6-10 for those choices
    if cfg["lik_mode"] in (0, 2):
        bound = H.ell_tolerance if cfg["lik_mode"] == 0 else H.ell_tolerance_poisson
        ref, tl, chosen = H.select_branches(cfg, frame, tr, g["ell"], bound,
                                            (tol[0], tol[1], tol[4]), k_done + 1)
    else:
        d = np.hypot(tr["prop"][0] - np.repeat(frame[:, 0], M * n_p),
                     tr["prop"][1] - np.repeat(frame[:, 1], M * n_p))
        tl = (d * (tol[0] + tol[1]) / cfg["noise_sigma"] ** 2 * 1.25 + 1e-6 * (1 + d * d))
        ref, chosen = tr, np.zeros(N, np.int64)
    n_amb = int(np.count_nonzero(tr["amb"]))
    n_other = int(np.count_nonzero(chosen))
    assert n_other <= max(2, N // 1000)
    dl = np.abs(g["ell"] - ref["ell"])
    assert np.all(dl <= tl), float(np.max(dl - tl))
    # fixed-point weights and ancestors, every PE
    qm = orc.qmax(n_p)
    mism = 0
    for pe in range(F * M):
        sl = slice(pe * n_p, (pe + 1) * n_p)
        tlam = 1e-6 * (1 + np.abs(tr["lambda"][sl]))
        tu = tl[sl] + tlam
        w = ref["Q"][sl] / qm
        tq = qm * w * (tu + tu.max()) * 1.01 + 2
        assert np.all(np.abs(g["q"][sl].astype(np.int64) - ref["Q"][sl].astype(np.int64)) <= tq)
        f, m = divmod(pe, M)
        mism += H.check_ancestors(g["q"][sl], g["v"][f, m], g["ancestors"][sl], ref["Q"][sl],
                                  ref["V"][f, m], ref["anc"][sl], tq)
    assert mism <= max(2, N // 200)
    # estimates, every PE, within 1e-4, or, for PEs of a few particles, within
    # what the weight tolerances allow: a weight error du_i moves x^m by
    # sum w_i du_i |x_i - x^m| / sum w_i (both sides, plus the coordinate
    # tolerance); global within 1e-4
    rec = g["pe_records"]
    u = (tr["lambda"] + ref["ell"]).reshape(F * M, n_p)
    w = np.exp(u - u.max(axis=1, keepdims=True))
    du = (tl + 1e-6 * (1 + np.abs(tr["lambda"]))).reshape(F * M, n_p)
    xo = tr["prop"].reshape(5, F * M, n_p)
    xm = ref["xhat_pe"].reshape(F * M, 5).T
    bound = (2 * (w * du * np.abs(xo - xm[:, :, None])).sum(axis=2) / w.sum(axis=1)
             + tol.reshape(5, F * M, n_p).max(axis=2)).T.reshape(F, M, 5)
    err = np.abs(rec[:, :, 1:6] - ref["xhat_pe"])
    assert np.all(err <= np.maximum(1e-4, bound)), float(err.max())
    assert np.allclose(g["est"]["x_global"], ref["xhat"], rtol=0, atol=1e-4)
    # log masses: log-sum-exp moves by at most the weight-averaged error of
    # its arguments, so a PE's L^(m) within the mean of its particles'
    # log-weight tolerances (or 1e-3)
    err_l = np.abs(rec[:, :, 0] - ref["L_pe"])
    bound_l = ((w * du).sum(axis=1) / w.sum(axis=1)).reshape(F, M)
    lim_l = np.maximum(1e-3, 1.01 * bound_l) + 1e-5 * np.abs(ref["L_pe"])
    print(f"  ambiguous patch centres {n_amb}, GPU on the other centre {n_other}, PEs "
          f"compared {F * M} of {F * M} (excluded 0), L_pe max err {err_l.max():.3g}, "
          f"log_z err {np.abs(g['est']['log_z_inc'] - ref['log_z']).max():.3g}", flush=True)
    assert np.all(err_l <= lim_l), float((err_l - lim_l).max())
    assert np.allclose(g["est"]["log_z_inc"], ref["log_z"], rtol=1e-5, atol=1e-3)
    assert np.allclose(g["est"]["pe_eff"], ref["pe_eff"], rtol=1e-4)
    check_next_nex(cfg, rec[:, :, 0], g["est"]["n_ex_next"], ref["n_ex_next"], lim_l)


def check_next_nex(cfg, L_gpu, nex_gpu, nex_orc, lim_l):
    """N_ex of the next iteration is an integer decided by floating point (the
    PE log-masses, through P_m = floor(exp(L_m - max L) 2^20)).  The device's
    value must be the exact rule (Eq. 3 and 4 in integers, the oracle's
    routine) applied to the device's own records.  The oracle's value comes
    from its own L_m, which differ within lim_l: a change of every L_m by at
    most d moves S^2 / D = PE_eff by a factor within exp(+-4 d), hence N_ex =
    N_p / 2 (1 - (PE_eff - 1) / (M - 1)) by at most N_p PE_eff (e^{4d} - 1) /
    (2 (M - 1)) + 1; across the cut-off (PE_eff > c M: no exchange) either
    side may be taken."""
    F, M, n_p = cfg["n_filters"], cfg["n_pe"], cfg["n_per_pe"]
    for f in range(F):
        L = L_gpu[f]
        if not np.isfinite(L.max()):
            continue
        P = np.floor(np.exp(L - L.max()) * 2.0 ** 20)
        want = orc.nex(P.astype(np.uint32), n_p, mode=cfg["mode"],
                       fixed_ratio=cfg["fixed_ratio"], initial_ratio=cfg["initial_ratio"],
                       cutoff=cfg["eff_cutoff"], first=False)
        assert int(nex_gpu[f]) == want, (f, int(nex_gpu[f]), want)
        if int(nex_gpu[f]) == int(nex_orc[f]):
            continue
        assert cfg["mode"] == 1 and M > 1, (f, int(nex_gpu[f]), int(nex_orc[f]))
        d = float(np.max(lim_l[f]))
        S = P.sum()
        eff = S * S / float((P * P).sum())
        grow = np.expm1(4 * d)
        bound = n_p * eff * grow / (2 * (M - 1)) + 1
        near_cut = abs(eff - cfg["eff_cutoff"] * M) <= eff * grow
        ok = abs(int(nex_gpu[f]) - int(nex_orc[f])) <= bound or (
            near_cut and 0 in (int(nex_gpu[f]), int(nex_orc[f])))
        assert ok, (f, int(nex_gpu[f]), int(nex_orc[f]), bound)


def test_master_step_of_many_pes():
    """With many PEs the last workgroup of each filter computes the master
    step once: the next iteration's N_ex equals the one the master step
    reports from the same records, and the carried weights are the records'
    log-masses renormalized by their log-sum-exp, over several iterations."""
    p = pf()
    cfg, frame, state, logmass = seeded_case("arna_2x2100x4")
    F, M = cfg["n_filters"], cfg["n_pe"]
    g = p.Tracker(cfg, np.zeros((F, 5), np.float32), debug=p.PF_DEBUG_TRACE)
    g.set_state(state, logmass, step=3)
    fr = torch.from_numpy(frame).cuda()
    prev = g.estimate()
    L_prev = logmass
    for it in range(4):
        g.step(fr)
        est = g.estimate()
        if it > 0:
            assert np.array_equal(est["n_ex"], prev["n_ex_next"]), it
        lam = g.debug_get("lam").reshape(F, M, -1)
        src = g.debug_get("src").reshape(F, M, -1) // cfg["n_per_pe"] % M
        for f in range(F):
            lse = np.logaddexp.reduce(L_prev[f])
            want = L_prev[f][src[f]] - lse
            assert np.allclose(lam[f], want, rtol=1e-6, atol=1e-5), (it, f)
        prev, L_prev = est, est["log_mass_pe"]
    g.close()


def test_exchange_map_export():
    p = pf()
    cfg, frame, state, logmass = seeded_case("arna_ragged_2x3x100")
    g = p.Tracker(cfg, np.zeros((2, 5), np.float32))
    g.set_state(state, logmass, step=4)
    src = torch.zeros(g.N, dtype=torch.int64, device="cuda")
    g.exchange(src)
    with pytest.raises(p.PFError):
        g.exchange(None)
    o = orc.Oracle(cfg, np.zeros((2, 5), np.float32))
    o.set_state(state.astype(np.float64), logmass, 4)
    tr = o.step(frame, want={"src_map"})
    assert np.array_equal(src.cpu().numpy(), tr["src_map"])
    g.step(torch.from_numpy(frame).cuda())   # steps 4-10 after the exported exchange
    g.close()


def test_exchange_map_export_streaming():
    """The source map of a context beyond the LDS stage (computed slot by
    slot) against the oracle's."""
    p = pf()
    cfg, frame, state, logmass = seeded_case("poisson_rna_1x2x20000")
    g = p.Tracker(cfg, np.zeros((1, 5), np.float32))
    g.set_state(state, logmass, step=2)
    src = torch.zeros(g.N, dtype=torch.int64, device="cuda")
    g.exchange(src)
    o = orc.Oracle(cfg, np.zeros((1, 5), np.float32))
    o.set_state(state.astype(np.float64), logmass, 2)
    tr = o.step(frame, want={"src_map"})
    assert np.array_equal(src.cpu().numpy(), tr["src_map"])
    g.close()


# ------------------------------------------------------------- multi-step runs
def test_rna_small_workload_end_to_end():
    p = pf()
    seq = synth.make_sequence("rna_128_4x256", seed=1000)
    cfg = synth.filter_config("rna_128_4x256", seed=3)
    truth0 = seq.initial_truth()[:1]
    g = p.Tracker(cfg, truth0, debug=p.PF_DEBUG_TRACE)
    o = orc.Oracle(cfg, truth0)
    frames = torch.from_numpy(seq.frames).cuda()
    eg, eo = [], []
    for k in range(1, seq.frames.shape[0] + 1):
        g.step(frames[k - 1])
        est = g.estimate()
        tr = o.step(seq.frames[k - 1], want={"xhat", "n_ex", "ring_pred"})
        assert est["step"] == k
        assert int(est["n_ex"][0]) == int(tr["n_ex"][0]) == 25
        assert np.array_equal(g.debug_get("ring"), tr["ring_pred"])
        if k == 1:
            assert np.allclose(est["x_global"], tr["xhat"], atol=1e-4, rtol=0)
        assert np.abs(est["x_global"][0, :2] - tr["xhat"][0, :2]).max() < 0.15
        eg.append(est["x_global"][0, :2] - seq.truth[k, 0, :2])
        eo.append(tr["xhat"][0, :2] - seq.truth[k, 0, :2])
    g.close()
    assert np.sqrt(np.mean(np.square(eg))) < 0.5
    assert np.sqrt(np.mean(np.square(eo))) < 0.5


def test_determinism_and_resume_bitwise():
    p = pf()
    seq = synth.make_sequence("rna_128_4x256", seed=1001, frames=8)
    cfg = synth.filter_config("rna_128_4x256", seed=11, mode=1, n_pe=8, n_per_pe=300)
    truth0 = seq.initial_truth()[:1]
    frames = torch.from_numpy(seq.frames).cuda()

    def run(n, tr=None):
        t = tr or p.Tracker(cfg, truth0)
        t.run(frames[:n])
        return t

    a = run(8)
    b = run(8)
    sa, sb = a.debug_get("state"), b.debug_get("state")
    assert np.array_equal(sa, sb)
    assert np.array_equal(a.debug_get("pe_records"), b.debug_get("pe_records"))
    c = run(4)
    st, L = c.debug_get("state"), c.debug_get("logmass")
    c.close()
    d = p.Tracker(cfg, truth0)
    d.set_state(st, L, step=4)
    d.run(frames[4:8])
    assert np.array_equal(d.debug_get("state"), sa)
    assert np.array_equal(d.debug_get("logmass"), a.debug_get("logmass"))
    for t in (a, b, d):
        t.close()


def test_infoshare_init_parity():
    p = pf()
    cfg = synth.filter_config("arna_infoshare_512_256x4096", n_pe=16, n_per_pe=512, seed=5)
    truth = np.array([[200.3, 300.6, 1.0, -0.5, 8.0]], np.float32)
    g = p.Tracker(cfg, truth)
    st = g.debug_get("state")
    g.close()
    o = orc.Oracle(cfg, truth)
    so, L, k = o.get_state()
    assert k == 0 and np.all(L == 0)
    for c in range(5):
        assert np.all(np.abs(st[c] - so[c]) <= H.coord_tol(so[c]))


def test_edge_single_pe_single_particle_and_full_exchange():
    p = pf()
    rng = np.random.Generator(np.random.PCG64(9))
    frame = synth.render(np.array([[20.0, 20.0, 0, 0, 10.0]]), 40, 40, 1.5, 5.0, 2.0, rng)
    ft = torch.from_numpy(frame).cuda()
    for over in [dict(n_pe=1, n_per_pe=64, mode=1), dict(n_pe=3, n_per_pe=1, mode=0,
                                                        fixed_ratio=1.0),
                 dict(n_pe=4, n_per_pe=50, mode=0, fixed_ratio=1.0),
                 dict(n_pe=3, n_per_pe=1, mode=0, fixed_ratio=1.0, pes_per_wg=2),
                 dict(n_pe=4, n_per_pe=50, mode=0, fixed_ratio=1.0, pes_per_wg=4),
                 dict(n_pe=2, n_per_pe=4097, mode=0, fixed_ratio=1.0),
                 dict(n_pe=1, n_per_pe=6000, mode=1)]:
        cfg = dict(n_filters=1, width=40, height=40, patch=9, init_mode=0, lik_mode=0,
                   initial_ratio=0.1, eff_cutoff=0.99, psf_sigma=1.5, background=5.0,
                   noise_sigma=2.0, q=0.5, sigma_I=0.5, seed=21, fixed_ratio=0.1)
        cfg.update(over)
        truth = np.array([[20.0, 20.0, 0.0, 0.0, 10.0]], np.float32)
        g = p.Tracker(cfg, truth, debug=p.PF_DEBUG_TRACE)
        o = orc.Oracle(cfg, truth)
        g.step(ft)
        est = g.estimate()
        tr = o.step(frame)
        assert np.array_equal(g.debug_get("src"), tr["src_map"])
        assert int(est["n_ex"][0]) == int(tr["n_ex"][0])
        assert np.allclose(est["x_global"], tr["xhat"], atol=1e-4, rtol=0)
        g.close()


def test_nan_pixel_sets_sticky_numeric_error():
    p = pf()
    frame = np.full((40, 40), 5.0, np.float32)
    frame[20, 20] = np.nan
    cfg = dict(n_filters=1, n_pe=2, n_per_pe=64, width=40, height=40, seed=2)
    g = p.Tracker(cfg, np.array([[20.0, 20.0, 0, 0, 10.0]], np.float32))
    g.step(torch.from_numpy(frame).cuda())
    with pytest.raises(p.PFError) as ei:
        g.estimate()
    assert ei.value.code == -4
    g.step(torch.from_numpy(np.full((40, 40), 5.0, np.float32)).cuda())
    assert g.estimate(raise_numeric=False)["status"] == -4   # sticky
    g.close()


@pytest.mark.parametrize("n_p,over", [(64, {}), (64, dict(pes_per_wg=2)), (5000, {})])
def test_dead_pe_gets_no_mass(n_p, over):
    """A PE without mass (L = -inf) keeps none: one PE per workgroup, several
    PEs per workgroup, split PEs."""
    p = pf()
    cfg = dict(n_filters=1, n_pe=4, n_per_pe=n_p, width=40, height=40, seed=2, mode=0,
               fixed_ratio=0.0, **over)
    rng = np.random.Generator(np.random.PCG64(4))
    state = synth.random_state(rng, 1, 4, n_p, 40, 40, spread=1.0, centre=[[20, 20]])
    L = np.array([[0.0, -np.inf, 0.0, 0.0]])
    g = p.Tracker(cfg, np.zeros((1, 5), np.float32))
    g.set_state(state, L, step=3)
    frame = synth.render(np.array([[20.0, 20.0, 0, 0, 10.0]]), 40, 40, 1.5, 5.0, 2.0, rng)
    g.step(torch.from_numpy(frame).cuda())
    est = g.estimate()
    o = orc.Oracle(cfg, np.zeros((1, 5), np.float32))
    o.set_state(state.astype(np.float64), L, 3)
    tr = o.step(frame, want={"L_pe", "xhat", "pe_eff"})
    assert est["log_mass_pe"][0, 1] == -np.inf and tr["L_pe"][0, 1] == -np.inf
    assert np.allclose(est["x_global"], tr["xhat"], atol=1e-4, rtol=0)
    assert est["pe_eff"][0] <= 3.0 + 1e-9
    g.close()


# --------------------------------------------------------- information spread
def lineage_run(mode, M, n_p, steps):
    p = pf()
    cfg = dict(n_filters=1, n_pe=M, n_per_pe=n_p, width=64, height=64, mode=mode,
               lik_mode=1, fixed_ratio=0.5, initial_ratio=0.5, eff_cutoff=1.0,
               noise_sigma=3.0, seed=4242)
    g = p.Tracker(cfg, np.array([[32.0, 32.0, 0.0, 0.0, 5.0]], np.float32),
                  debug=p.PF_DEBUG_LINEAGE | p.PF_DEBUG_TRACE)
    g.set_lineage(np.repeat(np.arange(M), n_p))
    z = torch.tensor([[32.0, 32.0]], dtype=torch.float32, device="cuda")
    infected, rings = [{0}], []
    for k in range(steps):
        g.step(z)
        tags = g.debug_get("lineage").reshape(M, n_p)
        infected.append({m for m in range(M) if np.any(tags[m] == 0)})
        rings.append(g.debug_get("ring")[0].copy())
    g.close()
    return infected, rings


def test_gpu_fixed_ring_confines_lineage():
    infected, _ = lineage_run(0, 12, 32, 8)
    for k, inf in enumerate(infected):
        assert inf <= set(range(k + 1))


def test_gpu_random_ring_infection_at_most_doubles():
    infected, rings = lineage_run(1, 32, 32, 8)
    for k in range(1, len(infected)):
        pred = rings[k - 1]
        reach = infected[k - 1] | {m for m in range(32) if int(pred[m]) in infected[k - 1]}
        assert infected[k] <= reach


# ---------------------------------------------- Philox against rocRAND (P8)
def test_oracle_philox_matches_rocrand_host_generator():
    """rocRAND's PHILOX4_32_10 run as a black box (its host generator needs a
    HIP device to allocate, so this test needs a GPU)."""
    import os
    path = "/opt/rocm/lib/librocrand.so"
    lib = ctypes.CDLL(path if os.path.exists(path) else "librocrand.so")
    gen = ctypes.c_void_p()
    if lib.rocrand_create_generator_host_blocking(ctypes.byref(gen), 404) != 0:
        pytest.skip("rocRAND host generator unavailable")
    seed = 0x0123456789ABCDEF
    assert lib.rocrand_set_seed(gen, ctypes.c_ulonglong(seed)) == 0
    n = 4096
    out = np.zeros(n, np.uint32)
    st = lib.rocrand_generate(gen, out.ctypes.data_as(ctypes.c_void_p), ctypes.c_size_t(n))
    lib.rocrand_destroy_generator(gen)
    assert st == 0
    key = [seed & 0xFFFFFFFF, seed >> 32]
    blocks = {tuple(orc.philox([i, 0, 0, 0], key)) for i in range(n // 4)}
    got = {tuple(out[4 * i:4 * i + 4]) for i in range(n // 4)}
    assert got == blocks
