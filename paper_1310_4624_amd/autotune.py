"""Workgroup-size autotuner: for a filter configuration, time the candidate
workgroup sizes (multiples of 64 up to 1024 that give every PE 1, 2 or 4
slots per thread) on the GPU path and keep the fastest.

Results are cached per shape (N_p, M, F, frame, patch, likelihood, mode) in
memory and, if a path is given, in a JSON file.  Every candidate computes the
same iteration; only the speed differs (a different workgroup size changes
nothing in the results but the order of floating-point sums).
"""
from __future__ import annotations

import json
import os

import numpy as np

from . import _native as nat
from .tracker import Tracker

_CACHE: dict = {}


def candidates(n_p: int) -> list:
    """Workgroup sizes worth timing for N_p particles per PE: the powers of two
    from 64 and N_p rounded up to 64, at most that and 1024, and large
    enough that 4 slots per thread cover N_p (PEs beyond the LDS stage: the
    streaming kernel's 1024 only)."""
    if n_p > nat.PF_MAX_PER_PE_LDS:
        return [1024]
    top = min(1024, (n_p + 63) // 64 * 64)
    sizes = {b for b in (64, 128, 256, 512, 1024) if b <= top} | {top}
    return sorted(b for b in sizes if 4 * b >= n_p)


def _key(cfg: dict) -> str:
    return "n_p={n_per_pe},M={n_pe},F={n_filters},{width}x{height},patch={patch},lik={lik_mode},mode={mode}".format(**cfg)


def tune(cfg: dict, truth, frames, steps: int = 6, cache_path: str | None = None) -> int:
    """The fastest block size for cfg; frames: CUDA float32 [K][...] with
    K >= steps + 2 (two warm-up iterations)."""
    import torch
    key = _key(cfg)
    if key in _CACHE:
        return _CACHE[key]
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as fh:
            disk = json.load(fh)
        if key in disk:
            _CACHE[key] = int(disk[key]["block_size"])
            return _CACHE[key]
    best, best_ms, times = None, None, {}
    for b in candidates(int(cfg["n_per_pe"])):
        tr = Tracker(dict(cfg, block_size=b), truth)
        tr.run(frames[:2])
        ms = float(np.median(tr.run_timed(frames[2:2 + steps])))
        tr.close()
        times[b] = ms
        if best_ms is None or ms < best_ms:
            best, best_ms = b, ms
    torch.cuda.synchronize()
    _CACHE[key] = best
    if cache_path:
        disk = {}
        if os.path.exists(cache_path):
            with open(cache_path) as fh:
                disk = json.load(fh)
        disk[key] = {"block_size": best, "ms": times}
        with open(cache_path, "w") as fh:
            json.dump(disk, fh, indent=1)
    return best
