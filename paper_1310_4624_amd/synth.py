"""Seeded synthetic inputs for the tracker: frame sequences, ground truth and
random test arrays.

This module only draws inputs.  It holds none of the filter's arithmetic and
imports neither the GPU binding nor the oracle, so both sides of a parity test
can take their inputs from it.

Frames stand in for the benchmark sequences of Sec. V (512 x 512 fluorescence
microscopy frames with small bright spots, Fig. 1), which are not available:
pixel = B + sum_spots I0 exp(-d^2 / (2 s^2)) + sigma_n N(0, 1), stored as float32.
Spot trajectories follow the nearly-constant-velocity model with a small
acceleration noise q_true (constant velocity for the small workload); start
boxes and speeds keep the spots away from the image margin over the sequence
(a reflection at the margin would be a velocity jump no NCV filter follows).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

MODE_RNA, MODE_ARNA = 0, 1
INIT_TRACKING, INIT_INFOSHARE = 0, 1
LIK_PATCH, LIK_POINT, LIK_POISSON = 0, 1, 2

def poisson_intensity(snr: float, background: float) -> float:
    """Peak intensity I0 with I0 / sqrt(B + I0) = snr (signal over the noise
    standard deviation at the spot's peak), for Poisson pixel noise."""
    return float(0.5 * (snr * snr + np.sqrt(snr ** 4 + 4.0 * snr * snr * background)))


# Workloads.  Each entry gives the filter configuration (keys shared by the GPU
# binding and the oracle) and the recipe of its synthetic sequence.
WORKLOADS = {
    # Plain RNA, CPU-sized: 1 spot, 128^2, 20 frames, 4 PEs x 256 particles.
    "rna_128_4x256": dict(
        filter=dict(n_filters=1, n_pe=4, n_per_pe=256, width=128, height=128, patch=9,
                    mode=MODE_RNA, init_mode=INIT_TRACKING, lik_mode=LIK_PATCH,
                    fixed_ratio=0.1, initial_ratio=0.1, eff_cutoff=0.99,
                    psf_sigma=1.5, background=5.0, noise_sigma=2.0, q=0.5, sigma_I=0.5),
        seq=dict(width=128, height=128, frames=20, intensities=[20.0], motion="constant",
                 speed=(1.0, 1.0), start_box=(40.0, 88.0), margin=16.0, min_sep=24.0),
    ),
    # ARNA tracking: 4 spots of SNR 2..6, 512^2, 100 frames, 4 filters x 64 PEs x 4096.
    "arna_tracking_512_4x64x4096": dict(
        filter=dict(n_filters=4, n_pe=64, n_per_pe=4096, width=512, height=512, patch=9,
                    mode=MODE_ARNA, init_mode=INIT_TRACKING, lik_mode=LIK_PATCH,
                    fixed_ratio=0.1, initial_ratio=0.1, eff_cutoff=0.99,
                    psf_sigma=1.5, background=5.0, noise_sigma=2.0, q=0.5, sigma_I=0.5),
        seq=dict(width=512, height=512, frames=100,
                 intensities=[2.0 * s for s in np.linspace(2.0, 6.0, 4)], motion="ncv",
                 speed=(0.5, 1.0), start_box=(160.0, 352.0), margin=16.0, min_sep=24.0,
                 q_true=0.001),
    ),
    # ARNA information sharing: 1 spot of SNR 4, 512^2, 200 frames, 256 PEs x 4096.
    "arna_infoshare_512_256x4096": dict(
        filter=dict(n_filters=1, n_pe=256, n_per_pe=4096, width=512, height=512, patch=9,
                    mode=MODE_ARNA, init_mode=INIT_INFOSHARE, lik_mode=LIK_PATCH,
                    fixed_ratio=0.1, initial_ratio=0.1, eff_cutoff=0.99,
                    psf_sigma=1.5, background=5.0, noise_sigma=2.0, q=0.5, sigma_I=0.5),
        seq=dict(width=512, height=512, frames=200, intensities=[8.0], motion="ncv",
                 speed=(0.3, 0.6), start_box=(192.0, 320.0), margin=16.0, min_sep=24.0,
                 q_true=0.001),
    ),
    # Poisson pixel noise (the noise of the paper's synthetic images), CPU-sized:
    # 1 spot of SNR 3.7 (I0 = 20 over B = 10 counts), 128^2, RNA 4 x 256.
    "rna_128_4x256_poisson": dict(
        filter=dict(n_filters=1, n_pe=4, n_per_pe=256, width=128, height=128, patch=9,
                    mode=MODE_RNA, init_mode=INIT_TRACKING, lik_mode=LIK_POISSON,
                    fixed_ratio=0.1, initial_ratio=0.1, eff_cutoff=0.99,
                    psf_sigma=1.5, background=10.0, noise_sigma=1.0, q=0.5, sigma_I=0.5),
        seq=dict(width=128, height=128, frames=20, intensities=[20.0], motion="constant",
                 speed=(1.0, 1.0), start_box=(40.0, 88.0), margin=16.0, min_sep=24.0,
                 noise="poisson"),
    ),
    # ARNA tracking with Poisson pixel noise: the tracking workload's shape,
    # 4 spots of Poisson SNR 2..6 over B = 10 counts.
    "arna_tracking_512_4x64x4096_poisson": dict(
        filter=dict(n_filters=4, n_pe=64, n_per_pe=4096, width=512, height=512, patch=9,
                    mode=MODE_ARNA, init_mode=INIT_TRACKING, lik_mode=LIK_POISSON,
                    fixed_ratio=0.1, initial_ratio=0.1, eff_cutoff=0.99,
                    psf_sigma=1.5, background=10.0, noise_sigma=1.0, q=0.5, sigma_I=0.5),
        seq=dict(width=512, height=512, frames=100,
                 intensities=[poisson_intensity(s, 10.0) for s in np.linspace(2.0, 6.0, 4)],
                 motion="ncv",
                 speed=(0.5, 1.0), start_box=(160.0, 352.0), margin=16.0, min_sep=24.0,
                 q_true=0.001, noise="poisson"),
    ),
    # The tracking workload scaled to 2^24 particles: 64 spots of SNR 2..6
    # (one filter each) x 64 PEs x 4096, 512^2, 40 frames.  Its state (2 x 320
    # MiB ping-pong) does not fit the 256 MB Infinity Cache.
    "arna_tracking_512_64x64x4096": dict(
        filter=dict(n_filters=64, n_pe=64, n_per_pe=4096, width=512, height=512, patch=9,
                    mode=MODE_ARNA, init_mode=INIT_TRACKING, lik_mode=LIK_PATCH,
                    fixed_ratio=0.1, initial_ratio=0.1, eff_cutoff=0.99,
                    psf_sigma=1.5, background=5.0, noise_sigma=2.0, q=0.5, sigma_I=0.5),
        seq=dict(width=512, height=512, frames=40,
                 intensities=[2.0 * s for s in np.linspace(2.0, 6.0, 64)], motion="ncv",
                 speed=(0.5, 1.0), start_box=(48.0, 464.0), margin=16.0, min_sep=24.0,
                 q_true=0.001, windowed=True),
    ),
    # Differentiable run: the information-sharing shape (256 PEs x 4096, 512^2,
    # one spot of SNR 4) over 50 frames, every particle starting at the truth,
    # so that the intensity gradient is the one of the true initial intensity.
    "arna_grad_512_256x4096": dict(
        filter=dict(n_filters=1, n_pe=256, n_per_pe=4096, width=512, height=512, patch=9,
                    mode=MODE_ARNA, init_mode=INIT_TRACKING, lik_mode=LIK_PATCH,
                    fixed_ratio=0.1, initial_ratio=0.1, eff_cutoff=0.99,
                    psf_sigma=1.5, background=5.0, noise_sigma=2.0, q=0.5, sigma_I=0.5),
        seq=dict(width=512, height=512, frames=50, intensities=[8.0], motion="ncv",
                 speed=(0.3, 0.6), start_box=(192.0, 320.0), margin=16.0, min_sep=24.0,
                 q_true=0.001),
    ),
}


@dataclass
class Sequence:
    frames: np.ndarray   # [K][H][W] float32; frames[k-1] is z_k
    truth: np.ndarray    # [K+1][S][5] float64; truth[k] is the state at step k
    spots: int

    def initial_truth(self) -> np.ndarray:
        """[S][5] float32 state at step 0, the pf_init / oracle truth argument."""
        return self.truth[0].astype(np.float32)


def _start_positions(rng, n, lo, hi, min_sep):
    pts = []
    for _ in range(10000):
        p = rng.uniform(lo, hi, size=2)
        if all(np.hypot(*(p - q)) >= min_sep for q in pts):
            pts.append(p)
            if len(pts) == n:
                return np.array(pts)
    raise RuntimeError("could not place the spots")


def _reflect(p, v, lo, hi):
    for a in range(2):
        if p[a] < lo[a]:
            p[a] = 2 * lo[a] - p[a]
            v[a] = -v[a]
        elif p[a] > hi[a]:
            p[a] = 2 * hi[a] - p[a]
            v[a] = -v[a]
    return p, v


def trajectories(rng, n_spots, n_frames, width, height, intensities, motion, speed, start_box,
                 margin, min_sep, q=0.5):
    """Ground-truth states [K+1][S][5] (x, y, vx, vy, I)."""
    pos = _start_positions(rng, n_spots, start_box[0], start_box[1], min_sep)
    truth = np.zeros((n_frames + 1, n_spots, 5))
    lo = np.array([margin, margin])
    hi = np.array([width - 1 - margin, height - 1 - margin])
    for s in range(n_spots):
        sp = rng.uniform(speed[0], speed[1])
        th = rng.uniform(0.0, 2 * np.pi)
        p = pos[s].copy()
        v = np.array([sp * np.cos(th), sp * np.sin(th)])
        truth[0, s] = [p[0], p[1], v[0], v[1], intensities[s]]
        L = np.linalg.cholesky(q * np.array([[1 / 3, 1 / 2], [1 / 2, 1.0]]))
        for k in range(1, n_frames + 1):
            if motion == "constant":
                p = p + v
            else:
                w = L @ rng.standard_normal((2, 2))   # column a = axis a
                p = p + v + w[0]
                v = v + w[1]
            p, v = _reflect(p, v, lo, hi)
            truth[k, s] = [p[0], p[1], v[0], v[1], intensities[s]]
    return truth


def render(truth_k, width, height, psf_sigma, background, noise_sigma, rng):
    """One frame: background + Gaussian spots + Gaussian pixel noise."""
    ys, xs = np.mgrid[0:height, 0:width].astype(np.float64)
    img = np.full((height, width), float(background))
    for s in range(truth_k.shape[0]):
        x, y, _, _, I0 = truth_k[s]
        img += I0 * np.exp(-((xs - x) ** 2 + (ys - y) ** 2) / (2 * psf_sigma ** 2))
    img += noise_sigma * rng.standard_normal((height, width))
    return img.astype(np.float32)


def render_poisson(truth_k, width, height, psf_sigma, background, rng):
    """One frame of photon counts: Poisson(B + sum_spots I0 exp(-d^2/(2 s^2)))."""
    ys, xs = np.mgrid[0:height, 0:width].astype(np.float64)
    lam = np.full((height, width), float(background))
    for s in range(truth_k.shape[0]):
        x, y, _, _, I0 = truth_k[s]
        lam += I0 * np.exp(-((xs - x) ** 2 + (ys - y) ** 2) / (2 * psf_sigma ** 2))
    return rng.poisson(lam).astype(np.float32)


def make_sequence(workload: str, seed: int = 1000, frames: int | None = None,
                  q_true: float | None = None) -> Sequence:
    """Frames and truth for a named workload (sequence seeds 1000.. by convention);
    q_true overrides the process noise of the true trajectories."""
    w = WORKLOADS[workload]
    sq, fl = w["seq"], w["filter"]
    K = sq["frames"] if frames is None else frames
    rng = np.random.Generator(np.random.PCG64(seed))
    q = q_true if q_true is not None else sq.get("q_true", fl["q"])
    truth = trajectories(rng, len(sq["intensities"]), K, sq["width"], sq["height"],
                         sq["intensities"], sq["motion"], sq["speed"], sq["start_box"],
                         sq["margin"], sq["min_sep"], q=q)
    out = np.zeros((K, sq["height"], sq["width"]), np.float32)
    for k in range(1, K + 1):
        if sq.get("noise") == "poisson":
            out[k - 1] = render_poisson(truth[k], sq["width"], sq["height"], fl["psf_sigma"],
                                        fl["background"], rng)
        else:
            draw = render_windowed if sq.get("windowed") else render
            out[k - 1] = draw(truth[k], sq["width"], sq["height"], fl["psf_sigma"],
                              fl["background"], fl["noise_sigma"], rng)
    return Sequence(frames=out, truth=truth, spots=len(sq["intensities"]))


def filter_config(workload: str, **overrides) -> dict:
    d = dict(WORKLOADS[workload]["filter"])
    d.update(overrides)
    return d


# ---------------------------------------------------------- batched sequences
def render_windowed(truth_k, width, height, psf_sigma, background, noise_sigma, rng, reach=8):
    """Like render(), with each spot evaluated only within `reach` px of its
    centre (its profile is below 1e-6 of the peak beyond 8 px at s = 1.5)."""
    img = np.full((height, width), float(background))
    for s in range(truth_k.shape[0]):
        x, y, _, _, I0 = truth_k[s]
        u0, u1 = max(int(np.floor(x)) - reach, 0), min(int(np.floor(x)) + reach + 1, width)
        v0, v1 = max(int(np.floor(y)) - reach, 0), min(int(np.floor(y)) + reach + 1, height)
        if u0 >= u1 or v0 >= v1:
            continue
        ys, xs = np.mgrid[v0:v1, u0:u1].astype(np.float64)
        img[v0:v1, u0:u1] += I0 * np.exp(-((xs - x) ** 2 + (ys - y) ** 2) / (2 * psf_sigma ** 2))
    img += noise_sigma * rng.standard_normal((height, width))
    return img.astype(np.float32)


def batch_sequences(seed: int = 2000, n_seq: int = 64, frames: int = 50):
    """Independent tracking problems of uneven size for the batched launch:
    frames of 256^2, 512^2 or 1024^2, 1-3 spots of SNR 2-8 (one filter per
    spot), 2^14..2^20 particles (log-uniform) over 16..256 PEs (log-uniform),
    so N_p = N / (F M) spans 64..65536 (at least 64; PEs above 4096 particles
    run the streaming step).  Returns [(cfg, truth [F][5] float32, frames
    [K][H][W])]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for i in range(n_seq):
        side = int(rng.choice([256, 512, 1024]))
        F = int(rng.integers(1, 4))
        N = int(round(2 ** rng.uniform(14, 20)))
        M = int(round(2 ** rng.uniform(4, 8)))
        n_p = max(64, N // (F * M))
        snr = rng.uniform(2.0, 8.0, F)
        cfg = dict(n_filters=F, n_pe=M, n_per_pe=n_p, width=side, height=side, patch=9,
                   mode=MODE_ARNA, init_mode=INIT_TRACKING, lik_mode=LIK_PATCH,
                   fixed_ratio=0.1, initial_ratio=0.1, eff_cutoff=0.99, psf_sigma=1.5,
                   background=5.0, noise_sigma=2.0, q=0.5, sigma_I=0.5, seed=1 + i)
        lo, hi = 0.3 * side, 0.7 * side
        truth = trajectories(rng, F, frames, side, side, list(2.0 * snr), "ncv", (0.3, 1.0),
                             (lo, hi), 16.0, 12.0, q=0.001)
        fr = np.stack([render_windowed(truth[k], side, side, 1.5, 5.0, 2.0, rng)
                       for k in range(1, frames + 1)])
        out.append((cfg, truth[0].astype(np.float32), fr))
    return out


# ----------------------------------------------------------------- small cases
def point_sequence(seed, n_filters, n_frames, q=0.5, r=1.0, start=(64.0, 64.0), I0=10.0):
    """Linear-Gaussian case: NCV truth (no reflection) and noisy position
    observations.  Returns (truth [K+1][F][5], obs [K][F][2] float32)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    L = np.linalg.cholesky(q * np.array([[1 / 3, 1 / 2], [1 / 2, 1.0]]))
    truth = np.zeros((n_frames + 1, n_filters, 5))
    obs = np.zeros((n_frames, n_filters, 2), np.float32)
    for f in range(n_filters):
        p = np.array(start, dtype=np.float64) + rng.uniform(-4, 4, 2)
        v = rng.uniform(-1, 1, 2)
        truth[0, f] = [p[0], p[1], v[0], v[1], I0]
        for k in range(1, n_frames + 1):
            w = L @ rng.standard_normal((2, 2))
            p = p + v + w[0]
            v = v + w[1]
            truth[k, f] = [p[0], p[1], v[0], v[1], I0]
            obs[k - 1, f] = p + np.sqrt(r) * rng.standard_normal(2)
    return truth, obs


def random_weights_q(rng, n_p, qmax, kind="mixed"):
    """Fixed-point weights Q in [0, qmax] with a mix of shapes (zeros, spikes,
    uniform, exponential tails); at least one entry equals qmax."""
    if kind == "uniform":
        Q = np.full(n_p, qmax, np.uint64)
    elif kind == "spike":
        Q = np.zeros(n_p, np.uint64)
    else:
        e = np.exp(-rng.exponential(3.0, n_p) * rng.uniform(0.1, 3.0))
        e[rng.random(n_p) < 0.2] = 0.0
        Q = np.floor(e * qmax).astype(np.uint64)
    Q[rng.integers(0, n_p)] = qmax
    return Q.astype(np.uint32)


def random_state(rng, n_filters, n_pe, n_per_pe, width, height, spread=3.0, centre=None,
                 I0=10.0):
    """A [5][N] float32 particle cloud around per-filter centres."""
    N = n_filters * n_pe * n_per_pe
    st = np.zeros((5, N), np.float32)
    for f in range(n_filters):
        sl = slice(f * n_pe * n_per_pe, (f + 1) * n_pe * n_per_pe)
        c = centre[f] if centre is not None else rng.uniform(16, [width - 16, height - 16])
        n = n_pe * n_per_pe
        st[0, sl] = c[0] + spread * rng.standard_normal(n)
        st[1, sl] = c[1] + spread * rng.standard_normal(n)
        st[2, sl] = rng.uniform(-2, 2, n)
        st[3, sl] = rng.uniform(-2, 2, n)
        st[4, sl] = I0 + rng.standard_normal(n)
    return st
