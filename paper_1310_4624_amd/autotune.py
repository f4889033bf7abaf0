"""Launch-shape autotuner: for a filter configuration, time the candidate
launch shapes on the GPU path and keep the fastest.  A shape has two axes:
the workgroup size (multiples of 64 up to 1024 that give every PE 1, 2 or 4
slots per thread) and the PEs per workgroup (1, or 2..16 PEs of a filter
sharing a workgroup, each on its own group of whole waves: the
particles-per-workgroup axis, which pays for small N_p).

Results are cached per shape (N_p, M, F, frame, patch, likelihood, mode) in
memory and, if a path is given, in a JSON file.  Every candidate computes the
same iteration; only the speed differs (a different shape changes nothing in
the results but the order of floating-point sums).
"""
from __future__ import annotations

import json
import os

import numpy as np

from . import _native as nat
from .tracker import Tracker

_CACHE: dict = {}


def candidates(n_p: int) -> list:
    """Workgroup sizes worth timing for N_p particles per PE with one PE per
    workgroup: the powers of two from 64 and N_p rounded up to 64, at most
    that and 1024, and large enough that 4 slots per thread cover N_p (PEs
    beyond the LDS stage: the streaming kernel's 1024 only)."""
    if n_p > nat.PF_MAX_PER_PE_LDS:
        return [1024]
    top = min(1024, (n_p + 63) // 64 * 64)
    sizes = {b for b in (64, 128, 256, 512, 1024) if b <= top} | {top}
    return sorted(b for b in sizes if 4 * b >= n_p)


def shapes(n_p: int, n_pe: int) -> list:
    """Launch shapes (block_size, pes_per_wg) worth timing: one PE per
    workgroup at every size of candidates(), and P = 2, 4, 8, 16 PEs per
    workgroup (P <= M) with N_p rounded up to 64 threads per PE (one slot per
    thread) and with the fewest threads that hold N_p in 4 slots each."""
    out = [(b, 1) for b in candidates(n_p)]
    if n_p > nat.PF_MAX_PER_PE_LDS:
        return out
    for ppw in (2, 4, 8, 16):
        if ppw > n_pe:
            break
        cap = 1024 // ppw // 64 * 64
        for tp in sorted({min(cap, (n_p + 63) // 64 * 64), max(64, (n_p + 255) // 256 * 64)}):
            if 64 <= tp <= cap and 4 * tp >= n_p:
                out.append((ppw * tp, ppw))
    return out


def _key(cfg: dict) -> str:
    return "n_p={n_per_pe},M={n_pe},F={n_filters},{width}x{height},patch={patch},lik={lik_mode},mode={mode}".format(**cfg)


def tune(cfg: dict, truth, frames, steps: int = 6, cache_path: str | None = None) -> dict:
    """The fastest launch shape for cfg, as config overrides
    {"block_size": B, "pes_per_wg": P}; frames: CUDA float32 [K][...] with
    K >= steps + 2 (two warm-up iterations)."""
    import torch
    key = _key(cfg)
    if key in _CACHE:
        return dict(_CACHE[key])
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as fh:
            disk = json.load(fh)
        if key in disk and "pes_per_wg" in disk[key]:
            _CACHE[key] = {"block_size": int(disk[key]["block_size"]),
                           "pes_per_wg": int(disk[key]["pes_per_wg"])}
            return dict(_CACHE[key])
    best, best_ms, times = None, None, {}
    for b, ppw in shapes(int(cfg["n_per_pe"]), int(cfg["n_pe"])):
        shape = {"block_size": b, "pes_per_wg": ppw}
        tr = Tracker(dict(cfg, **shape), truth)
        tr.run(frames[:2])
        ms = float(np.median(tr.run_timed(frames[2:2 + steps])))
        tr.close()
        times[f"{b}x{ppw}"] = ms
        if best_ms is None or ms < best_ms:
            best, best_ms = shape, ms
    torch.cuda.synchronize()
    _CACHE[key] = best
    if cache_path:
        disk = {}
        if os.path.exists(cache_path):
            with open(cache_path) as fh:
                disk = json.load(fh)
        disk[key] = dict(best, ms=times)
        with open(cache_path, "w") as fh:
            json.dump(disk, fh, indent=1)
    return dict(best)
