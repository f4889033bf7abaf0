"""Throughput of the ARNA SIR step on one MI355X.

A step is one full iteration of the hot path (ring, exchange ratio, exchange,
renormalization, propagation, patch likelihood, per-PE reductions, systematic
resampling, PE records) over all particles of the workload, frames already
resident in HBM.  Prints one JSON line.

Default workload: the ARNA tracking configuration, 4 filters x 64 PEs x 4096
particles (2^20 particles), 512 x 512 frames with 4 spots of SNR 2..6.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "particle-steps/s, full ARNA SIR step at 2^20 particles; fwd+bwd/fwd cost ratio"
HBM_PEAK_GBS = 8000.0
# Algorithmic HBM bytes per particle-step: read the float32 state (5 x 4 B),
# write the resampled state (5 x 4 B), and the frame (H W 4 B) shared by the
# N particles; the exchange is a read-index remap and moves no extra bytes.
STATE_BYTES = 40.0


def algorithmic_bytes(n_particles: int, width: int, height: int) -> float:
    return STATE_BYTES * n_particles + 4.0 * width * height


def gpu_leg(workload: str, steps: int, warmup: int, seed: int):
    import torch
    from paper_1310_4624_amd import Tracker, synth

    cfg = synth.filter_config(workload, seed=seed)
    seq = synth.make_sequence(workload, seed=1000, frames=warmup + steps)
    F = cfg["n_filters"]
    truth0 = seq.initial_truth()[:F]
    torch.cuda.set_device(0)
    frames = torch.from_numpy(seq.frames).cuda()
    stream = torch.cuda.current_stream()
    tr = Tracker(cfg, truth0)
    if warmup:
        tr.run(frames[:warmup])
    torch.cuda.synchronize()
    # per-step HIP events on the stream the kernels are launched on
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    t0 = time.perf_counter()
    ev[0].record(stream)
    for i in range(steps):
        tr.step(frames[warmup + i])
        ev[i + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    total_ms = ev[0].elapsed_time(ev[steps])
    per = np.array([ev[i].elapsed_time(ev[i + 1]) for i in range(steps)])
    est = tr.estimate()
    tr.close()
    # iterations k = 1, 65, 129, ... also build the next 64 rings (ARNA)
    ks = warmup + 1 + np.arange(steps)
    ring_steps = (ks - 1) % 64 == 0 if cfg["mode"] == 1 else np.zeros(steps, bool)
    step_ms = float(per[~ring_steps].mean()) if (~ring_steps).any() else float(per.mean())
    return dict(cfg=cfg, seq=seq, total_ms=total_ms, wall_s=wall, step_kernel_ms=step_ms,
                per_step_ms=per.tolist(), pe_eff=est["pe_eff"].tolist(),
                n_ex=est["n_ex"].tolist())


def cpu_leg(workload: str, seed: int, budget_s: float, seq):
    """The FP64 oracle on the host cores: whole iterations of the same
    workload on the same frames until the time budget is used (at least one)."""
    from oracle import oracle as orc
    from paper_1310_4624_amd import synth

    cfg = synth.filter_config(workload, seed=seed)
    F = cfg["n_filters"]
    o = orc.Oracle(cfg, seq.initial_truth()[:F])
    N = F * cfg["n_pe"] * cfg["n_per_pe"]
    done, t = 0, 0.0
    while done < seq.frames.shape[0] and (done == 0 or t < budget_s):
        t0 = time.perf_counter()
        o.step(seq.frames[done], trace=False)
        t += time.perf_counter() - t0
        done += 1
    return dict(value=N * done / t, unit="particle-steps/s", cores=orc.num_threads(),
                kind="oracle",
                sample=f"{workload}: first {done} iteration(s) of the same sequence, "
                       f"{N} particles, FP64, {t:.1f} s")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="arna_tracking_512_4x64x4096")
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for {args.gpus}); the "
              "multi-GPU sharding of the path is a design note, not code", file=sys.stderr)
        sys.exit(2)

    g = gpu_leg(args.workload, args.steps, args.warmup, args.seed)
    cfg = g["cfg"]
    N = cfg["n_filters"] * cfg["n_pe"] * cfg["n_per_pe"]
    ms = g["total_ms"] / args.steps
    value = N * args.steps / (g["total_ms"] / 1e3)
    bytes_launch = algorithmic_bytes(N, cfg["width"], cfg["height"])
    achieved = bytes_launch / (g["step_kernel_ms"] / 1e3) / 1e9
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "n_particles": N, "n_filters": cfg["n_filters"],
                   "n_pe": cfg["n_pe"], "n_per_pe": cfg["n_per_pe"],
                   "frame": f"{cfg['width']}x{cfg['height']}", "patch": cfg["patch"],
                   "mode": "ARNA" if cfg["mode"] == 1 else "RNA",
                   "parallelism": "one PE per workgroup, 1 GPU"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "k_step", "kernel_ms": g["step_kernel_ms"],
                     "bytes_per_launch": bytes_launch},
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_leg(args.workload, args.seed, args.cpu_budget, g["seq"])
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
