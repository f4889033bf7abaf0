"""Comparison helpers for the GPU-versus-oracle parity tests.

Tolerances follow from the arithmetic of the two sides (FP32 on the GPU, FP64
in the oracle) started from the same float32 inputs:
  * a propagated coordinate takes two float32 roundings of values of its own
    magnitude plus the error of the float32 normals (native log2, sqrt and
    sin/cos, relative error of a few 1e-7 on |eps| < 6): |dx| <= 2 ulp(x) + 1e-5;
  * a log-likelihood differs by the effect of those position errors (bounded
    with the likelihood's gradient over the patch) plus the float32 rounding of
    its 81-term sums, taken as 2e-6 of the sum of the magnitudes of its terms;
  * a fixed-point weight Q = floor(exp(u - lstar) Q_max) then moves by at most
    Q_max w (du + dlstar) + 2.
Particles whose oracle position lies within the coordinate tolerance of a
pixel boundary (x + 1/2 an integer) may sit on different patches on the two
sides: both patch centres are valid outcomes of the nearest-pixel decision.
The oracle reports the likelihood at the other centre(s) for such particles;
the comparison takes the one the GPU value agrees with, and the oracle
recomputes the per-PE and master steps for that choice (``select_branches``).
"""
from __future__ import annotations

import numpy as np

import oracle.oracle as orc


def ulp32(x):
    return np.spacing(np.abs(np.asarray(x, dtype=np.float32))).astype(np.float64)


def coord_tol(x, extra=1e-5):
    return 2.0 * ulp32(np.maximum(np.abs(x), 1.0)) + extra


def patch_flip_mask(x, y, tol_x, tol_y):
    fx = np.mod(np.asarray(x) + 0.5, 1.0)
    fy = np.mod(np.asarray(y) + 0.5, 1.0)
    return (fx < tol_x) | (fx > 1 - tol_x) | (fy < tol_y) | (fy > 1 - tol_y)


# The rounding a coordinate may carry on the GPU side (coord_tol) plus the
# float32 rounding of x + 1/2 in the nearest-pixel decision, as the ambiguity
# window of the oracle: eps_rel max(|x|, 1) + eps_abs.
AMB_EPS_REL = 4.0 * 2.0 ** -23
AMB_EPS_ABS = 2e-5


def ell_tolerance(cfg: dict, frame: np.ndarray, prop: np.ndarray, tol_x, tol_y, tol_I,
                  cx=None, cy=None):
    """Per-particle bound on |l_gpu - l_oracle| for patch mode (prop: [5][n]),
    with the patch centred at (cx, cy) (default: the nearest pixel)."""
    x, y, I = prop[0], prop[1], prop[4]
    half = cfg["patch"] // 2
    H, W = frame.shape
    s2 = cfg["psf_sigma"] ** 2
    sn2 = cfg["noise_sigma"] ** 2
    B = cfg["background"]
    cx = np.floor(x + 0.5) if cx is None else np.asarray(cx, np.float64)
    cy = np.floor(y + 0.5) if cy is None else np.asarray(cy, np.float64)
    gx_abs_sum = np.zeros_like(x)
    gy_abs_sum = np.zeros_like(x)
    ggx = np.zeros_like(x)
    ggy = np.zeros_like(x)
    sum_gz = np.zeros_like(x)
    sum_g2 = np.zeros_like(x)
    sum_abs_gz = np.zeros_like(x)
    ok = np.isfinite(cx) & np.isfinite(cy) & (np.abs(cx) < 1e8) & (np.abs(cy) < 1e8)
    cxi = np.where(ok, cx, -10 ** 6).astype(np.int64)
    cyi = np.where(ok, cy, -10 ** 6).astype(np.int64)
    for dv in range(-half, half + 1):
        v = cyi + dv
        for du in range(-half, half + 1):
            u = cxi + du
            inb = (u >= 0) & (u < W) & (v >= 0) & (v < H)
            z = np.where(inb, frame[np.clip(v, 0, H - 1), np.clip(u, 0, W - 1)], 0.0) - B
            z = np.where(inb, z, 0.0)
            ddx = u - x
            ddy = v - y
            g = np.where(inb, np.exp(-(ddx * ddx + ddy * ddy) / (2 * s2)), 0.0)
            dgx = g * np.abs(ddx) / s2
            dgy = g * np.abs(ddy) / s2
            gx_abs_sum += dgx * np.abs(z)
            gy_abs_sum += dgy * np.abs(z)
            ggx += g * dgx
            ggy += g * dgy
            sum_gz += g * z
            sum_g2 += g * g
            sum_abs_gz += np.abs(g * z)
    Gx = (np.abs(I) * gx_abs_sum + I * I * ggx) / sn2
    Gy = (np.abs(I) * gy_abs_sum + I * I * ggy) / sn2
    GI = np.abs(sum_gz - I * sum_g2) / sn2
    mag = (np.abs(I) * sum_abs_gz + 0.5 * I * I * sum_g2) / sn2
    # the gradient bound is taken at the oracle position; 25% margin for its
    # change over the (sub-1e-3 px) distance
    return 1.25 * (Gx * tol_x + Gy * tol_y + GI * tol_I) + 2e-6 * mag + 1e-6


def ell_tolerance_poisson(cfg: dict, frame: np.ndarray, prop: np.ndarray, tol_x, tol_y, tol_I,
                          cx=None, cy=None):
    """Per-particle bound on |l_gpu - l_oracle| for Poisson patch mode,
    l = sum [z log(1 + I g / B) - I g]: the gradient of l times the coordinate
    tolerances, plus FP32 rounding (the float log of 1 + t/B carries an
    absolute error of a few 1e-8 per pixel, times the count z)."""
    x, y, I = prop[0], prop[1], prop[4]
    half = cfg["patch"] // 2
    H, W = frame.shape
    s2 = cfg["psf_sigma"] ** 2
    B = cfg["background"]
    cx = np.floor(x + 0.5) if cx is None else np.asarray(cx, np.float64)
    cy = np.floor(y + 0.5) if cy is None else np.asarray(cy, np.float64)
    ok = np.isfinite(cx) & np.isfinite(cy) & (np.abs(cx) < 1e8) & (np.abs(cy) < 1e8)
    cxi = np.where(ok, cx, -10 ** 6).astype(np.int64)
    cyi = np.where(ok, cy, -10 ** 6).astype(np.int64)
    Gx = np.zeros_like(x)
    Gy = np.zeros_like(x)
    GI = np.zeros_like(x)
    mag = np.zeros_like(x)
    zsum = np.zeros_like(x)
    for dv in range(-half, half + 1):
        v = cyi + dv
        for du in range(-half, half + 1):
            u = cxi + du
            inb = (u >= 0) & (u < W) & (v >= 0) & (v < H)
            z = np.where(inb, frame[np.clip(v, 0, H - 1), np.clip(u, 0, W - 1)], 0.0)
            ddx, ddy = u - x, v - y
            g = np.where(inb, np.exp(-(ddx * ddx + ddy * ddy) / (2 * s2)), 0.0)
            lam = B + I * g
            dl_dg = np.abs(z * I / lam - I)
            Gx += dl_dg * g * np.abs(ddx) / s2
            Gy += dl_dg * g * np.abs(ddy) / s2
            GI += z * g / lam - g
            mag += np.abs(z * np.log1p(I * g / B)) + np.abs(I * g)
            zsum += z
    return 1.25 * (Gx * tol_x + Gy * tol_y + np.abs(GI) * tol_I) + 4e-6 * mag + 2e-7 * zsum + 1e-6


def check_ancestors(Qg, Vg, ancg, Qo, Vo, anco, tolQ):
    """Compare one PE's ancestors.  The GPU ancestors must be valid for the
    GPU's own fixed-point weights; where they differ from the oracle's, the
    pointer must lie within the weight tolerance of a cumulative boundary.
    Returns the number of explained mismatches."""
    n_p = len(Qg)
    Cg = np.cumsum(Qg.astype(np.int64))
    Tg = int(Cg[-1])
    ptr = np.arange(n_p, dtype=np.int64) * Tg + int(Vg)
    lo = np.where(ancg == 0, 0, n_p * Cg[np.maximum(ancg.astype(np.int64) - 1, 0)])
    hi = n_p * Cg[ancg]
    assert np.all((lo <= ptr) & (ptr < hi)), "GPU ancestors invalid for the GPU's own weights"
    mism = np.flatnonzero(ancg != anco)
    if len(mism) == 0:
        return 0
    Co = np.cumsum(Qo.astype(np.int64)).astype(np.float64)
    To = Co[-1]
    beta = Co / To
    rho = (np.arange(n_p) * To + Vo) / (n_p * To)
    eps = 2.0 * float(np.sum(tolQ)) / To + 4.0 / (n_p * To)
    for j in mism:
        a, b = sorted((int(ancg[j]), int(anco[j])))
        d = np.min(np.abs(rho[j] - beta[a:b]))
        assert d <= eps, (j, int(ancg[j]), int(anco[j]), d, eps)
    return len(mism)


def other_centre(x):
    """The other nearest-pixel candidate of a coordinate next to a boundary."""
    t = np.asarray(x) + 0.5
    b = np.floor(t + 0.5)
    c0 = np.floor(t)
    return np.where(c0 == b, b - 1.0, b)


def select_branches(cfg: dict, frame, tr: dict, ell_gpu, tol_fn, tol_xyI, k: int):
    """Oracle reference values for the patch-centre choices the GPU made.

    For every particle whose patch centre is ambiguous (oracle trace ``amb``),
    the candidate likelihoods are the oracle's own at its centre and at the
    other centre(s) (``ell_alt``); the candidate nearest the GPU value is
    taken (any of them is a valid outcome).  For every PE with a particle on
    another centre than the oracle's, the oracle reruns steps 6-7
    (``orc_pe_update``) with those likelihoods, and the master step 9-10
    (``orc_master``) of its filter is rerun.  Returns (ref, tl, chosen): ref
    holds the trace arrays with those replacements, tl the per-particle
    likelihood tolerance at the chosen centres, chosen the candidate index
    (0: the oracle's centre, 1: other x, 2: other y, 3: both)."""
    F, M, n_p = cfg["n_filters"], cfg["n_pe"], cfg["n_per_pe"]
    prop = tr["prop"]
    tol_x, tol_y, tol_I = tol_xyI
    ref = {key: np.array(v, copy=True) for key, v in tr.items() if isinstance(v, np.ndarray)}
    cand = np.concatenate([tr["ell"][:, None], tr["ell_alt"]], axis=1)
    dist = np.abs(cand - np.asarray(ell_gpu, np.float64)[:, None])
    dist[~np.isfinite(cand)] = np.inf
    chosen = np.argmin(dist, axis=1)
    ref["ell"] = cand[np.arange(len(chosen)), chosen]
    cx = np.floor(prop[0] + 0.5)
    cy = np.floor(prop[1] + 0.5)
    cx = np.where((chosen == 1) | (chosen == 3), other_centre(prop[0]), cx)
    cy = np.where((chosen == 2) | (chosen == 3), other_centre(prop[1]), cy)
    tl = np.zeros(len(chosen))
    for f in range(F):
        sl = slice(f * M * n_p, (f + 1) * M * n_p)
        tl[sl] = tol_fn(cfg, frame, prop[:, sl], tol_x[sl], tol_y[sl], tol_I[sl], cx[sl], cy[sl])
    moved = chosen.reshape(F * M, n_p) != 0
    for pe in np.flatnonzero(moved.any(axis=1)):
        f, m = divmod(int(pe), M)
        sl = slice(pe * n_p, (pe + 1) * n_p)
        r = orc.pe_update(cfg, f, k, m, tr["lambda"][sl], ref["ell"][sl], prop[:, sl])
        ref["Q"][sl] = r["Q"]
        ref["anc"][sl] = r["anc"]
        ref["T"][f, m] = r["T"]
        ref["V"][f, m] = r["V"]
        ref["L_pe"][f, m] = r["L_pe"]
        ref["lstar"][f, m] = r["lstar"]
        ref["xhat_pe"][f, m] = r["xhat_pe"]
    for f in sorted({int(pe) // M for pe in np.flatnonzero(moved.any(axis=1))}):
        g = orc.master(cfg, ref["L_pe"][f], ref["xhat_pe"][f])
        ref["xhat"][f] = g["xhat"]
        ref["L_glob"][f] = g["L_glob"]
        ref["P"][f] = g["P"]
        ref["pe_eff"][f] = g["pe_eff"]
        ref["log_z"][f] = g["log_z"]
        ref["n_ex_next"][f] = g["n_ex_next"]
    return ref, tl, chosen
