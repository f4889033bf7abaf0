"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: published
known-answer vectors, closed forms, exact rational arithmetic, brute force on
tiny inputs, distributional facts, or an independently written plain SIR.
"""
import math
import os
from fractions import Fraction

import numpy as np
import pytest
from scipy import stats

import oracle.oracle as orc
from oracle.kalman import kalman_means
from paper_1310_4624_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
SEED = 0x1234_5678_9ABC
KEY = [SEED & 0xFFFFFFFF, SEED >> 32]


# ----------------------------------------------------------------- Philox (P8)
def load_kat():
    rows = []
    with open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            v = [int(t, 16) for t in line.split()]
            rows.append((v[0:4], v[4:6], v[6:10]))
    return rows


def test_philox_known_answer_vectors():
    rows = load_kat()
    assert len(rows) == 3
    for ctr, key, want in rows:
        assert list(orc.philox(ctr, key)) == want


def test_philox_word_uniformity():
    words = np.concatenate([orc.philox([i, 7, 0, 4 << 24], KEY) for i in range(6000)])
    top = (words >> 24).astype(np.int64)
    counts = np.bincount(top, minlength=256)
    assert stats.chisquare(counts).pvalue > 1e-4
    bits = np.array([(words >> b) & 1 for b in range(32)]).mean(axis=1)
    assert np.all(np.abs(bits - 0.5) < 5 * 0.5 / np.sqrt(words.size))


def test_five_normals_distribution():
    n = 12000
    e = np.array([orc.normals(SEED, 0, 3, j) for j in range(n)])
    for c in range(5):
        x = e[:, c]
        assert abs(x.mean()) < 5 / np.sqrt(n)
        assert abs(x.var() - 1.0) < 5 * np.sqrt(2.0 / n)
        assert stats.kstest(x, "norm").pvalue > 1e-4
    corr = np.corrcoef(e.T)
    assert np.all(np.abs(corr - np.eye(5)) < 5 / np.sqrt(n))


# ----------------------------------------------------- systematic resampling (P1)
def interval_check(Q, V, anc):
    n_p = len(Q)
    C = np.cumsum(np.asarray(Q, dtype=np.int64))
    T = int(C[-1])
    for j, a in enumerate(anc):
        lo = 0 if a == 0 else n_p * int(C[a - 1])
        assert lo <= j * T + V < n_p * int(C[a])


@pytest.mark.parametrize("n_p", [1, 2, 3, 5, 8])
def test_systematic_brute_force(n_p):
    rng = np.random.Generator(np.random.PCG64(n_p))
    for trial in range(4):
        Q = rng.integers(0, 700, n_p).astype(np.uint32)
        Q[rng.integers(0, n_p)] = rng.integers(1, 700)
        T = int(Q.astype(np.int64).sum())
        total = np.zeros(n_p, dtype=np.int64)
        for V in range(T):
            anc = orc.resample(Q, V)
            assert np.all(np.diff(anc.astype(np.int64)) >= 0)
            cnt = np.bincount(anc, minlength=n_p)
            assert cnt.sum() == n_p
            for i in range(n_p):
                lo = (n_p * int(Q[i])) // T
                hi = -((-n_p * int(Q[i])) // T)
                assert lo <= cnt[i] <= hi
            if V % 37 == 0:
                interval_check(Q, V, anc)
            total += cnt
        # unbiasedness as an integer identity: sum over all offsets of the
        # offspring count of i is exactly N_p Q_i
        assert np.array_equal(total, n_p * Q.astype(np.int64))


def test_systematic_uniform_weights_is_identity():
    for n_p in [1, 7, 64, 256]:
        Q = np.full(n_p, orc.qmax(n_p), np.uint32)
        T = int(Q.astype(np.int64).sum())
        for V in [0, 1, T // 3, T - 1]:
            assert np.array_equal(orc.resample(Q, V), np.arange(n_p))


def test_systematic_single_mass():
    Q = np.zeros(50, np.uint32)
    Q[17] = 12345
    for V in [0, 5000, 12344]:
        assert np.all(orc.resample(Q, V) == 17)


def test_systematic_rejects_bad_offset():
    with pytest.raises(ValueError):
        orc.resample(np.array([3, 4], np.uint32), 7)
    with pytest.raises(ValueError):
        orc.resample(np.zeros(4, np.uint32), 0)


def test_qmax_keeps_totals_in_32_bits():
    for n_p in [1, 2, 3, 255, 256, 257, 4096, 65535]:
        qm = orc.qmax(n_p)
        assert qm <= 1 << 24
        assert qm * n_p <= 0xFFFFFFFF


# ------------------------------------------------------------------- ring (P3)
@pytest.mark.parametrize("M", [1, 2, 3, 5, 16, 257])
def test_ring_is_single_cycle(M):
    for k in range(1, 30):
        pi, pred, succ = orc.ring(SEED, 0, k, M)
        assert sorted(pi.tolist()) == list(range(M))
        assert np.array_equal(pred[succ], np.arange(M))
        seen, node = set(), 0
        for hop in range(M):
            seen.add(node)
            node = int(succ[node])
        assert node == 0 and len(seen) == M


def test_rna_ring_is_fixed_neighbour():
    M = 11
    for k in [1, 2, 50]:
        pi, pred, succ = orc.ring(SEED, 0, k, M, mode=orc.MODE_RNA)
        assert np.array_equal(succ, (np.arange(M) + 1) % M)
        assert np.array_equal(pred, (np.arange(M) - 1) % M)


def test_fisher_yates_uniform_over_permutations():
    import itertools
    perms = {p: i for i, p in enumerate(itertools.permutations(range(4)))}
    counts = np.zeros(24, dtype=np.int64)
    for k in range(1, 12001):
        pi, _, _ = orc.ring(SEED, 0, k, 4)
        counts[perms[tuple(pi.tolist())]] += 1
    assert stats.chisquare(counts).pvalue > 1e-4


def test_ring_differs_between_steps_and_filters():
    a = orc.ring(SEED, 0, 5, 64)[0]
    b = orc.ring(SEED, 0, 6, 64)[0]
    c = orc.ring(SEED, 1, 5, 64)[0]
    assert not np.array_equal(a, b) and not np.array_equal(a, c)


# ------------------------------------------------------------ exchange ratio (P4)
def eq3_exact(P, n_p, cutoff=Fraction(99, 100)):
    M = len(P)
    S = sum(int(p) for p in P)
    D = sum(int(p) * int(p) for p in P)
    pe_eff = Fraction(S * S, D)
    if pe_eff > cutoff * M:
        return 0
    val = n_p * (Fraction(1, 2) - Fraction(1, 2) * (pe_eff - 1) / (M - 1))
    return math.floor(val)


def test_nex_equal_masses_is_zero():
    for M in [2, 7, 64, 256]:
        P = np.full(M, 1 << 20, np.uint32)
        assert orc.nex(P, 4096) == 0
        assert orc.nex(P, 4096, cutoff=1.0) == 0


def test_nex_one_pe_holds_everything():
    for M in [2, 3, 64, 256]:
        P = np.zeros(M, np.uint32)
        P[M // 2] = 1 << 20
        for n_p in [1, 7, 256, 4096]:
            assert orc.nex(P, n_p) == n_p // 2


def test_nex_k_equal_masses_gives_pe_eff_k():
    M, n_p = 24, 4096
    for kk in range(1, M + 1):
        P = np.zeros(M, np.uint32)
        P[:kk] = 777
        want = 0 if kk > 0.99 * M else (n_p * (M - kk)) // (2 * (M - 1))
        assert orc.nex(P, n_p) == want


def test_nex_cutoff_boundary():
    n_p = 4096
    P = np.full(100, 1 << 20, np.uint32)
    P[99] = 0                          # PE_eff = 99 = 0.99 M exactly: not above
    assert orc.nex(P, n_p) == (n_p * 99) // (2 * 99 * 99) == n_p // 198
    P[99] = 1                          # PE_eff just above 0.99 M: no exchange
    assert orc.nex(P, n_p) == 0


def test_nex_matches_exact_rational_eq3():
    rng = np.random.Generator(np.random.PCG64(3))
    for trial in range(300):
        M = int(rng.integers(2, 400))
        n_p = int(rng.integers(1, 10000))
        P = np.floor(np.exp(-rng.exponential(rng.uniform(0.1, 8), M)) * 2 ** 20).astype(np.uint32)
        P[rng.integers(0, M)] = 1 << 20
        assert orc.nex(P, n_p) == eq3_exact(P, n_p), (M, n_p)


def test_nex_large_M_no_overflow():
    rng = np.random.Generator(np.random.PCG64(4))
    M = 65535
    P = rng.integers(0, (1 << 20) + 1, M).astype(np.uint32)
    P[0] = 1 << 20
    for n_p in [4096, 65535]:
        assert orc.nex(P, n_p, cutoff=1.0) == eq3_exact(P, n_p, cutoff=Fraction(2))


def test_nex_modes_and_degenerate_cases():
    P = np.array([1 << 20, 5, 0, 9], np.uint32)
    assert orc.nex(P, 256, mode=orc.MODE_RNA, fixed_ratio=0.1) == 25
    assert orc.nex(P, 256, mode=orc.MODE_RNA, fixed_ratio=0.5) == 128
    assert orc.nex(P, 256, mode=orc.MODE_RNA, fixed_ratio=0.0) == 0
    assert orc.nex(P, 4096, first=True, initial_ratio=0.1) == 409
    assert orc.nex(P[:1], 4096) == 0                     # M = 1
    assert orc.fixed_nex(0.1, 256) == 25


# ----------------------------------------------------------- exchange map (P2)
def run_one_step(M, n_p, ratio, mode=orc.MODE_RNA, seed=5, k0=0):
    cfg = dict(n_filters=2, n_pe=M, n_per_pe=n_p, width=64, height=64, mode=mode,
               lik_mode=orc.LIK_POINT, fixed_ratio=ratio, initial_ratio=ratio, seed=seed)
    o = orc.Oracle(cfg, np.tile([32.0, 32.0, 0.5, 0.5, 10.0], (2, 1)))
    return o.step(np.array([[32.0, 32.0], [31.0, 33.0]], np.float32)), o.cfg


@pytest.mark.parametrize("M,n_p,ratio", [(4, 16, 0.25), (5, 10, 0.5), (3, 7, 0.3),
                                         (8, 64, 1.0), (1, 8, 0.5), (6, 33, 0.1)])
def test_exchange_map_is_ring_permutation(M, n_p, ratio):
    tr, cfg = run_one_step(M, n_p, ratio)
    N = cfg.N
    src = tr["src_map"]
    assert np.array_equal(np.sort(src), np.arange(N))
    for f in range(2):
        n_ex = int(tr["n_ex"][f])
        assert n_ex == (0 if M == 1 else orc.fixed_nex(ratio, n_p))
        pred = tr["ring_pred"][f]
        for m in range(M):
            g = (f * M + m) * n_p + np.arange(n_p)
            sp = src[g] // n_p - f * M
            moved = sp != m
            if M > 1:
                assert moved.sum() == n_ex
                assert np.all(sp[moved] == pred[m])
                assert np.array_equal(src[g][~moved], g[~moved])
                # received particles land in the slots this PE sent away
                sent = sorted(orc.selected_slot(t, int(tr["exch_off"][f][m]), n_p, n_ex)
                              for t in range(n_ex))
                assert np.flatnonzero(moved).tolist() == sent
            else:
                assert not moved.any()


def test_exchange_selection_distinct_and_fair():
    n_p, n_ex, keys = 40, 7, 6000
    freq = np.zeros(n_p)
    for k in range(1, keys + 1):
        c = orc.exchange_offset(SEED, 0, k, 3, n_p)
        assert 0 <= c < n_p
        sel = [orc.selected_slot(t, c, n_p, n_ex) for t in range(n_ex)]
        assert len(set(sel)) == n_ex and max(sel) < n_p
        freq[sel] += 1
    p = n_ex / n_p
    assert np.all(np.abs(freq / keys - p) < 5 * np.sqrt(p * (1 - p) / keys))


# ------------------------------------------------------------- likelihood (P6)
LIK = dict(n_filters=1, n_pe=1, n_per_pe=1, width=48, height=40, patch=9, psf_sigma=1.5,
           background=5.0, noise_sigma=2.0)


def spot_image(x, y, I0, w=48, h=40, s=1.5, B=5.0):
    ys, xs = np.mgrid[0:h, 0:w].astype(np.float64)
    return B + I0 * np.exp(-((xs - x) ** 2 + (ys - y) ** 2) / (2 * s * s))


def test_loglik_noise_free_closed_form():
    x, y, I0 = 20.3, 17.8, 12.0
    img = spot_image(x, y, I0).astype(np.float32)
    cx, cy = math.floor(x + 0.5), math.floor(y + 0.5)
    gx = sum(math.exp(-((u - x) ** 2) / (2 * 1.5 ** 2)) ** 2 for u in range(cx - 4, cx + 5))
    gy = sum(math.exp(-((v - y) ** 2) / (2 * 1.5 ** 2)) ** 2 for v in range(cy - 4, cy + 5))
    want = I0 * I0 * gx * gy / (2 * 2.0 ** 2)
    # float32 frame: the residual is below the float32 rounding of the pixels
    got = orc.loglik(LIK, img, 0, [x, y, 0, 0, I0])
    assert abs(got - want) < 1e-4 * want


def test_loglik_maximum_at_truth():
    x, y, I0 = 20.2, 17.1, 10.0
    img = spot_image(x, y, I0).astype(np.float32)
    best = orc.loglik(LIK, img, 0, [x, y, 0, 0, I0])
    for dx in np.linspace(-0.25, 0.25, 6):
        for dy in np.linspace(-0.35, 0.35, 6):
            for dI in [-1.0, 0.0, 1.0]:
                if dx == 0 and dy == 0 and dI == 0:
                    continue
                assert orc.loglik(LIK, img, 0, [x + dx, y + dy, 0, 0, I0 + dI]) < best + 1e-9


@pytest.mark.parametrize("x,y", [(20.3, 17.8), (1.2, 2.7), (46.6, 39.4), (-3.0, 20.0),
                                 (50.9, 43.2), (0.5, 0.5), (-4.6, 5.0)])
def test_loglik_equals_full_image_gaussian_ratio(x, y):
    rng = np.random.Generator(np.random.PCG64(11))
    img = (spot_image(24.0, 20.0, 9.0) + 2.0 * rng.standard_normal((40, 48))).astype(np.float32)
    I = 7.5
    # patch indicator: pixels within 4 of the pixel nearest the particle
    cx, cy = math.floor(x + 0.5), math.floor(y + 0.5)
    ys, xs = np.mgrid[0:40, 0:48]
    inpatch = (np.abs(xs - cx) <= 4) & (np.abs(ys - cy) <= 4)
    g = np.exp(-((xs - x) ** 2 + (ys - y) ** 2) / (2 * 1.5 ** 2)) * inpatch
    z = img.astype(np.float64)
    logn_spot = -((z - 5.0 - I * g) ** 2) / (2 * 4.0)
    logn_bg = -((z - 5.0) ** 2) / (2 * 4.0)
    want = float(np.sum(logn_spot - logn_bg))
    got = orc.loglik(LIK, img, 0, [x, y, 0, 0, I])
    assert abs(got - want) < 1e-9 * max(1.0, abs(want))


def test_loglik_patch_far_outside_image_is_zero():
    img = np.zeros((40, 48), np.float32)
    for st in ([-100.0, 5, 0, 0, 5], [5, 1e9, 0, 0, 5], [np.inf, 3, 0, 0, 1]):
        assert orc.loglik(LIK, img, 0, st) == 0.0


def test_loglik_point_mode():
    cfg = dict(LIK, lik_mode=orc.LIK_POINT, noise_sigma=1.5)
    z = np.array([[10.0, 4.0]], np.float32)
    got = orc.loglik(cfg, z, 0, [11.0, 2.0, 0, 0, 0])
    assert got == pytest.approx(-(1.0 + 4.0) / (2 * 2.25), rel=1e-12)


# --------------------------------------------------------------- dynamics
def test_propagate_deterministic_part_and_unit_noise():
    s = [10.0, 20.0, 1.5, -0.5, 8.0]
    assert np.allclose(orc.propagate(s, np.zeros(5), 0.5, 0.5), [11.5, 19.5, 1.5, -0.5, 8.0],
                       atol=0, rtol=0)
    q = 0.5
    out = orc.propagate(s, [1.0, 0, 0, 0, 0], q, 0.5)
    assert out[0] == pytest.approx(11.5 + math.sqrt(q / 3))
    assert out[2] == pytest.approx(1.5 + math.sqrt(q) * math.sqrt(3) / 2)
    out = orc.propagate(s, [0, 1.0, 0, 0, 2.0], q, 0.5)
    assert out[0] == 11.5 and out[2] == pytest.approx(1.5 + math.sqrt(q) / 2)
    assert out[4] == pytest.approx(9.0)


def test_propagate_noise_covariance_is_white_acceleration():
    q = 0.8
    n = 20000
    e = np.array([orc.normals(SEED, 0, 9, j) for j in range(n)])
    s = np.array([0.0, 0.0, 0.0, 0.0, 0.0])
    d = np.array([orc.propagate(s, e[i], q, 0.3) for i in range(n)])
    cov = np.cov(d[:, [0, 2]].T)
    want = q * np.array([[1 / 3, 1 / 2], [1 / 2, 1.0]])
    assert np.allclose(cov, want, rtol=0.06, atol=0.01)
    assert np.var(d[:, 4]) == pytest.approx(0.09, rel=0.06)
    assert abs(np.corrcoef(d[:, 0], d[:, 1])[0, 1]) < 0.04


# ---------------------------------------------------- Kalman special case (P5)
@pytest.mark.parametrize("mode,ratio", [(orc.MODE_RNA, 0.0), (orc.MODE_RNA, 0.1),
                                        (orc.MODE_RNA, 0.5), (orc.MODE_ARNA, 0.1)])
def test_converges_to_kalman_mean(mode, ratio):
    F, K, q, r = 6, 8, 0.5, 1.0
    truth, obs = synth.point_sequence(21, F, K, q=q, r=r)
    kf = np.array([kalman_means(truth[0, f, :4], obs[:, f], q, r) for f in range(F)])
    sizes, errs = [], []
    for logn in [10, 12, 14, 16]:
        M = 4
        n_p = (1 << logn) // M
        cfg = dict(n_filters=F, n_pe=M, n_per_pe=n_p, width=128, height=128, mode=mode,
                   lik_mode=orc.LIK_POINT, fixed_ratio=ratio, initial_ratio=0.1, q=q,
                   noise_sigma=math.sqrt(r), sigma_I=0.5, seed=1000 + logn)
        o = orc.Oracle(cfg, truth[0].astype(np.float32))
        e2 = []
        for k in range(K):
            tr = o.step(obs[k], want={"xhat"})
            e2.append(np.sum((tr["xhat"][:, :2] - kf[:, k, :2]) ** 2, axis=1))
        sizes.append(1 << logn)
        errs.append(np.sqrt(np.mean(e2)))
    slope = np.polyfit(np.log(sizes), np.log(errs), 1)[0]
    assert -0.6 <= slope <= -0.4, (slope, errs)


# ---------------------------------------------- decomposition into plain SIR (P7)
def plain_sir(states, frame, k, m, n_p, f, seed, cfg):
    """Independent plain SIR (Alg. 1 with resampling at every step) of one PE,
    drawing from the same Philox counters as PE m of a multi-PE filter."""
    key = [seed & 0xFFFFFFFF, seed >> 32]
    sq = math.sqrt(cfg["q"])
    props, ells = [], []
    for s in range(n_p):
        r = [int(v) for v in orc.philox([m * n_p + s, k, f, 4 << 24], key)]
        u = [(2.0 * (v >> 9) + 1.0) / 2.0 ** 24 for v in r]
        ra = math.sqrt(-2 * math.log(u[0]))
        rb = math.sqrt(-2 * math.log(u[2]))
        uc = (2.0 * ((r[0] & 511) | ((r[1] & 511) << 9)) + 1.0) / 2.0 ** 19
        ud = (2.0 * ((r[2] & 511) | ((r[3] & 511) << 9)) + 1.0) / 2.0 ** 19
        e = [ra * math.cos(2 * math.pi * u[1]), ra * math.sin(2 * math.pi * u[1]),
             rb * math.cos(2 * math.pi * u[3]), rb * math.sin(2 * math.pi * u[3]),
             math.sqrt(-2 * math.log(uc)) * math.cos(2 * math.pi * ud)]
        x, y, vx, vy, I = states[s]
        nx = x + vx + sq * e[0] / math.sqrt(3)
        nvx = vx + sq * (math.sqrt(3) / 2 * e[0] + e[1] / 2)
        ny = y + vy + sq * e[2] / math.sqrt(3)
        nvy = vy + sq * (math.sqrt(3) / 2 * e[2] + e[3] / 2)
        nI = I + cfg["sigma_I"] * e[4]
        props.append([nx, ny, nvx, nvy, nI])
        cx, cy = math.floor(nx + 0.5), math.floor(ny + 0.5)
        ell = 0.0
        for v in range(cy - 4, cy + 5):
            for uu in range(cx - 4, cx + 5):
                if 0 <= v < frame.shape[0] and 0 <= uu < frame.shape[1]:
                    g = math.exp(-((uu - nx) ** 2 + (v - ny) ** 2) / (2 * cfg["psf_sigma"] ** 2))
                    z = float(frame[v, uu]) - cfg["background"]
                    ell += (2 * nI * g * z - nI * nI * g * g) / (2 * cfg["noise_sigma"] ** 2)
        ells.append(ell)
    ells = np.array(ells)
    w = np.exp(ells - ells.max())
    est = (w[:, None] * np.array(props)).sum(0) / w.sum()
    qm = orc.qmax(n_p)
    Q = np.floor(w * qm).astype(np.int64)
    T = int(Q.sum())
    V = (int(orc.philox([m, k, f, 5 << 24], key)[0]) * T) >> 32
    C = np.cumsum(Q)
    anc = [int(np.searchsorted(n_p * C, j * T + V, side="right")) for j in range(n_p)]
    return [props[a] for a in anc], anc, est, ells.max() + math.log(w.sum())


def test_single_pe_arna_is_plain_sir():
    cfg = dict(n_filters=1, n_pe=1, n_per_pe=48, width=40, height=36, mode=orc.MODE_ARNA,
               psf_sigma=1.5, background=5.0, noise_sigma=2.0, q=0.5, sigma_I=0.5, seed=77)
    rng = np.random.Generator(np.random.PCG64(5))
    truth0 = [18.0, 17.0, 0.7, -0.4, 11.0]
    o = orc.Oracle(cfg, np.array([truth0], np.float32))
    states = [list(np.float32(truth0).astype(np.float64))] * 48
    for k in range(1, 5):
        pos = (18.0 + 0.7 * k, 17.0 - 0.4 * k)
        frame = (spot_image(*pos, 11.0, w=40, h=36) + 2 * rng.standard_normal((36, 40))
                 ).astype(np.float32)
        tr = o.step(frame)
        states, anc, est, _ = plain_sir(states, frame, k, 0, 48, 0, 77, cfg)
        assert tr["n_ex"][0] == 0
        assert tr["anc"].tolist() == anc
        assert np.allclose(tr["state"].T, np.array(states), rtol=0, atol=1e-9)
        assert np.allclose(tr["xhat"][0], est, rtol=0, atol=1e-9)


def test_rna_zero_exchange_is_independent_pes():
    M, n_p = 3, 24
    cfg = dict(n_filters=1, n_pe=M, n_per_pe=n_p, width=40, height=36, mode=orc.MODE_RNA,
               fixed_ratio=0.0, psf_sigma=1.5, background=5.0, noise_sigma=2.0, q=0.5,
               sigma_I=0.5, seed=91)
    rng = np.random.Generator(np.random.PCG64(6))
    truth0 = [20.0, 15.0, -0.3, 0.6, 9.0]
    o = orc.Oracle(cfg, np.array([truth0], np.float32))
    pe_states = [[list(np.float32(truth0).astype(np.float64))] * n_p for _ in range(M)]
    L_carried = np.zeros(M)            # log W^(m)_{k-1}; all PEs start equal
    for k in range(1, 4):
        frame = (spot_image(20 - 0.3 * k, 15 + 0.6 * k, 9.0, w=40, h=36)
                 + 2 * rng.standard_normal((36, 40))).astype(np.float32)
        tr = o.step(frame)
        Ls, ests = [], []
        for m in range(M):
            pe_states[m], anc, est, Lm = plain_sir(pe_states[m], frame, k, m, n_p, 0, 91, cfg)
            assert tr["anc"][m * n_p:(m + 1) * n_p].tolist() == anc
            assert np.allclose(tr["xhat_pe"][0, m], est, atol=1e-9, rtol=0)
            Ls.append(Lm)
            ests.append(est)
        # W^(m)_k = W^(m)_{k-1} / W_{k-1} * sum_i p(z | x_i): the PE keeps its
        # carried mass; the master's estimate is the W-weighted mean
        lam = L_carried - (L_carried.max() + np.log(np.exp(L_carried - L_carried.max()).sum()))
        L_carried = lam + np.array(Ls)
        assert np.allclose(tr["L_pe"][0], L_carried, atol=1e-9, rtol=0)
        W = np.exp(L_carried - L_carried.max())
        assert np.allclose(tr["xhat"][0], (W[:, None] * np.array(ests)).sum(0) / W.sum(),
                           atol=1e-9, rtol=0)


# --------------------------------------------------- information spread (P11)
def lineage_run(mode, M, n_p, steps, ratio=0.5):
    cfg = dict(n_filters=1, n_pe=M, n_per_pe=n_p, width=64, height=64, mode=mode,
               lik_mode=orc.LIK_POINT, fixed_ratio=ratio, initial_ratio=0.5, eff_cutoff=1.0,
               noise_sigma=3.0, seed=4242)
    o = orc.Oracle(cfg, np.array([[32.0, 32.0, 0.0, 0.0, 5.0]], np.float32))
    o.set_lineage(np.repeat(np.arange(M), n_p))
    infected = [{0}]
    rings = []
    for k in range(steps):
        tr = o.step(np.array([[32.0, 32.0]], np.float32))
        tags = tr["lineage"].reshape(M, n_p)
        infected.append({m for m in range(M) if np.any(tags[m] == 0)})
        rings.append(tr["ring_pred"][0].copy())
    return infected, rings


def test_fixed_ring_confines_pe0_lineage():
    infected, _ = lineage_run(orc.MODE_RNA, 12, 32, 8)
    for k, inf in enumerate(infected):
        assert inf <= set(range(0, k + 1))


def test_random_ring_infection_at_most_doubles():
    infected, rings = lineage_run(orc.MODE_ARNA, 32, 32, 8)
    for k in range(1, len(infected)):
        pred = rings[k - 1]
        reach = infected[k - 1] | {m for m in range(32) if int(pred[m]) in infected[k - 1]}
        assert infected[k] <= reach
        assert len(infected[k]) <= 2 * len(infected[k - 1])


# ------------------------------------------------------------- accuracy (P10)
def test_small_rna_tracks_the_spot():
    seq = synth.make_sequence("rna_128_4x256", seed=1000)
    cfg = synth.filter_config("rna_128_4x256", seed=1)
    o = orc.Oracle(cfg, seq.initial_truth()[:1])
    err = []
    for k in range(1, seq.frames.shape[0] + 1):
        tr = o.step(seq.frames[k - 1], want={"xhat", "n_ex", "pe_eff"})
        assert tr["status"] == 0 and tr["n_ex"][0] == 25
        err.append(np.sum((tr["xhat"][0, :2] - seq.truth[k, 0, :2]) ** 2))
    assert np.sqrt(np.mean(err)) < 0.5
