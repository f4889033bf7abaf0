"""Throughput of the ARNA SIR step on one MI355X.

A step is one full iteration of the hot path (ring, exchange ratio, exchange,
renormalization, propagation, patch likelihood, per-PE reductions, systematic
resampling, PE records, and the master step: global estimate, W_k, PE_eff,
next N_ex and likelihood increment, written to a device trajectory buffer)
over all particles of the workload, frames already resident in HBM.  Prints
one JSON line.

Default workload: the ARNA tracking configuration, 4 filters x 64 PEs x 4096
particles (2^20 particles), 512 x 512 frames with 4 spots of SNR 2..6; the
information-sharing configuration (1 x 256 x 4096) is measured the same way
and reported beside it.

Timing: after the warm-up, one pf_run_traj of K steps (K = 64 by default, so
that an ARNA run rebuilds its ring table once inside the region) is bracketed
by two HIP events on the stream the kernels run on (the metric).  A second
region of steps, each bracketed by events that the library records on the same
stream around its step launch, gives the step kernel's average duration for
the roofline entry.
"""
from __future__ import annotations

import argparse
import hashlib
import re
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
# write the resampled state (5 x 4 B); plus the frame (H W 4 B) once per step,
# shared by all particles.  The exchange is a read-index remap and moves no
# extra bytes.
STATE_BYTES = 40.0
# the device code (kernels and their helpers); host-side changes keep the record
KERNEL_SOURCES = ["paper_1310_4624_amd/csrc/arna_kernels.hpp",
                  "paper_1310_4624_amd/csrc/arna_device.hpp"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_step_traffic.json")
HEADLINE = "arna_tracking_512_4x64x4096"
SECOND = "arna_infoshare_512_256x4096"


def algorithmic_bytes(n_particles: int, width: int, height: int) -> float:
    return STATE_BYTES * n_particles + 4.0 * width * height


def code_tokens(text: str) -> str:
    """C++ source without its comments and with runs of white space made one
    space (string literals in the kernel sources hold no comment markers)."""
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def kernel_sha() -> str:
    """Hash of the k_step sources' code (comments and layout excluded), which
    ties the stored counters to the kernel they were taken on."""
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), encoding="utf-8") as fh:
            h.update(code_tokens(fh.read()).encode())
    return h.hexdigest()[:16]


def measured_counters(workload: str, ring_groups: int = 0):
    """Counter summary of k_step (HBM bytes and VALU instructions per launch)
    from profiles/k_step_traffic.json, or None when the kernel sources changed
    since the counters were taken or the workload differs."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if (t.get("kernel_sha") != kernel_sha() or t.get("workload") != workload
            or t.get("ring_groups", 0) != ring_groups):
        return None
    return t


# VALU issue: 256 CUs x 4 SIMDs at 2.4 GHz, one wave64 instruction per SIMD
# every 4 cycles (16 lanes wide)
VALU_WAVE_INSTR_PER_S = 1024 * 2.4e9 / 4


def valu_entry(counters, kernel_ms: float, n_particles: int):
    """VALU use of k_step from the counters in profiles/k_step_traffic.json:
    instructions per particle-step, the instruction classes, and the busy
    fraction rocprofv3's VALUBusy reports (SQ_ACTIVE_INST_VALU, the cycles
    VALU instructions occupy -- so quarter-rate and transcendental
    instructions weigh what they cost -- per CU over GRBM_GUI_ACTIVE)."""
    if not counters or "valu_insts" not in counters:
        return None
    v = {"insts_per_launch": counters["valu_insts"],
         "insts_per_particle_step": counters["valu_insts"] * 64.0 / n_particles,
         "issue_ms_at_4_cycles": counters["valu_insts"] / VALU_WAVE_INSTR_PER_S * 1e3}
    if "valu_busy_pct" in counters:
        v["busy_frac"] = counters["valu_busy_pct"] / 100.0
    for k in ("valu_by_class", "wait_inst_any", "salu_insts", "lds_insts",
              "lds_bank_conflict_cycles"):
        if k in counters:
            v[k] = counters[k]
    return v


def gpu_leg(workload: str, steps: int, warmup: int, seed: int, probe: int, ring_groups: int = 0):
    import torch
    from paper_1310_4624_amd import Tracker, synth

    from paper_1310_4624_amd import TRAJ_RECORD_BYTES, trajectory

    cfg = synth.filter_config(workload, seed=seed, ring_groups=ring_groups)
    n_frames = max(warmup + 2 * steps + probe, synth.WORKLOADS[workload]["seq"]["frames"])
    seq = synth.make_sequence(workload, seed=1000, frames=n_frames)
    F = cfg["n_filters"]
    torch.cuda.set_device(0)
    frames = torch.from_numpy(seq.frames[:warmup + 2 * steps + probe]).cuda()
    traj = torch.empty(max(steps, 1) * F * TRAJ_RECORD_BYTES, dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()
    tr = Tracker(cfg, seq.initial_truth()[:F])
    if warmup:
        tr.run(frames[:warmup])
    torch.cuda.synchronize()

    # timed region: K steps in one call, every iteration's master step
    # written to the device trajectory, two events
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    tr.run_traj(frames[warmup:warmup + steps], traj)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    total_ms = e0.elapsed_time(e1)
    tj = trajectory(traj, steps, F)

    # context: the same number of steps without the per-iteration master
    # record (pf_run)
    e0.record(stream)
    tr.run(frames[warmup + steps:warmup + 2 * steps])
    e1.record(stream)
    torch.cuda.synchronize()
    plain_ms = e0.elapsed_time(e1)

    # kernel-duration region: the library records a pair of HIP events around
    # each step launch on the same stream (no host round trip in between)
    lo = warmup + 2 * steps
    per = tr.run_timed(frames[lo:lo + probe]).astype(np.float64)
    ks = lo + 1 + np.arange(probe)
    # iterations k = 1, 65, 129, ... also build the next 64 rings (ARNA)
    ring = (ks - 1) % 64 == 0 if cfg["mode"] == 1 else np.zeros(probe, bool)
    step_ms = float(per[~ring].mean()) if (~ring).any() else float(per.mean())
    tr.close()
    return dict(cfg=cfg, seq=seq, total_ms=total_ms, plain_ms=plain_ms, wall_s=wall,
                step_kernel_ms=step_ms, pe_eff=tj["pe_eff"][-1].tolist(),
                n_ex=tj["n_ex"][-1].tolist(), log_z_sum=tj["log_z_inc"].sum(0).tolist(),
                traj_steps=[int(tj["step"][0][0]), int(tj["step"][-1][0])] if steps else [])


def phase_leg(workload: str, seed: int, spread: int = 20, converged: int = 64):
    """The information-sharing workload from its start, in its two phases:
    iterations 1..spread, while the PEs are still spread over the frame (most
    patches read the frame), and the next `converged` iterations, once they
    share the spot (patches read the LDS tile).  Each phase is one pf_run_traj
    call between two events; a separate context loads the kernels first."""
    import torch
    from paper_1310_4624_amd import TRAJ_RECORD_BYTES, Tracker, synth

    cfg = synth.filter_config(workload, seed=seed)
    seq = synth.make_sequence(workload, seed=1000, frames=spread + converged)
    frames = torch.from_numpy(seq.frames).cuda()
    F = cfg["n_filters"]
    traj = torch.empty(max(spread, converged) * F * TRAJ_RECORD_BYTES, dtype=torch.uint8,
                       device="cuda")
    stream = torch.cuda.current_stream()
    warm = Tracker(cfg, seq.initial_truth()[:F])
    warm.run_traj(frames[:2], traj)
    warm.close()
    tr = Tracker(cfg, seq.initial_truth()[:F])
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    ev[0].record(stream)
    tr.run_traj(frames[:spread], traj)
    ev[1].record(stream)
    tr.run_traj(frames[spread:spread + converged], traj)
    ev[2].record(stream)
    torch.cuda.synchronize()
    tr.close()
    return {"spread_iterations": [1, spread],
            "spread_ms_per_step": ev[0].elapsed_time(ev[1]) / spread,
            "converged_iterations": [spread + 1, spread + converged],
            "converged_ms_per_step": ev[1].elapsed_time(ev[2]) / converged}


def grad_leg(workload: str, frames_n: int, seed: int):
    """Cost of the gradient: K iterations forward, then the same K iterations
    recorded plus the reverse sweep (pf_grad_end), on the same frames and
    start.  Both regions are bracketed by events on the library's stream;
    each is measured three times and the medians are reported."""
    import torch
    from paper_1310_4624_amd import Tracker, synth

    cfg = synth.filter_config(workload, seed=seed)
    seq = synth.make_sequence(workload, seed=1000, frames=frames_n)
    frames = torch.from_numpy(seq.frames).cuda()
    stream = torch.cuda.current_stream()
    truth = seq.initial_truth()[:cfg["n_filters"]]
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    # warm-up of both paths (kernel loading, tape allocation)
    tr = Tracker(cfg, truth)
    tr.grad_begin(frames_n)
    tr.run(frames[:2])
    tr.grad_end(frames[:2])
    tr.close()
    torch.cuda.synchronize()

    # three measurements of each region (a context made afresh each time);
    # the medians are reported
    fwds, boths = [], []
    for _ in range(3):
        tr = Tracker(cfg, truth)
        torch.cuda.synchronize()
        ev[0].record(stream)
        tr.run(frames)
        ev[1].record(stream)
        torch.cuda.synchronize()
        tr.close()
        tr = Tracker(cfg, truth)
        torch.cuda.synchronize()
        ev[2].record(stream)
        tr.grad_begin(frames_n)
        tr.run(frames)
        res = tr.grad_end(frames)
        ev[3].record(stream)
        torch.cuda.synchronize()
        tr.close()
        fwds.append(ev[0].elapsed_time(ev[1]))
        boths.append(ev[2].elapsed_time(ev[3]))
    fwd = sorted(fwds)[1]
    both = sorted(boths)[1]
    return {"workload": workload, "frames": frames_n,
            "n_particles": cfg["n_filters"] * cfg["n_pe"] * cfg["n_per_pe"],
            "fwd_ms": fwd, "fwd_bwd_ms": both, "fwd_bwd_over_fwd": both / fwd,
            "fwd_ms_runs": fwds, "fwd_bwd_ms_runs": boths,
            "J": res["J"].tolist(), "dJ_dtheta": res["grad"].tolist(),
            "theta": ["psf_sigma", "I0", "q"]}


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_leg(workload: str, seed: int, budget_s: float, seq, threads: int = 0):
    """The FP64 oracle on the host cores: whole iterations of the same
    workload on the same frames until the time budget is used (at least one),
    with `threads` OpenMP threads (0: the runtime's default).  When the frames
    run out before the budget, a new filter runs the sequence again from its
    start (at most four passes)."""
    from oracle import oracle as orc
    from paper_1310_4624_amd import synth

    default = orc.num_threads()
    orc.set_num_threads(threads or default)
    cfg = synth.filter_config(workload, seed=seed)
    F = cfg["n_filters"]
    K = seq.frames.shape[0]
    N = F * cfg["n_pe"] * cfg["n_per_pe"]
    done, t, passes, i, o = 0, 0.0, 0, K, None
    while done == 0 or t < budget_s:
        if i == K:
            if passes == 4:
                break
            o = orc.Oracle(cfg, seq.initial_truth()[:F])
            passes, i = passes + 1, 0
        t0 = time.perf_counter()
        o.step(seq.frames[i], trace=False)
        t += time.perf_counter() - t0
        i += 1
        done += 1
    used = orc.num_threads()
    orc.set_num_threads(default)
    return dict(value=N * done / t, unit="particle-steps/s", cores=used,
                kind="oracle",
                sample=f"{workload}: {done} iterations ({passes} pass(es) over the first "
                       f"{min(done, K)} frames of the same sequence), {N} particles, "
                       f"FP64, {t:.1f} s")


def main():
    from paper_1310_4624_amd import synth

    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=64)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--probe", type=int, default=20, help="single steps timed for the roofline")
    ap.add_argument("--workload", default=HEADLINE, choices=sorted(synth.WORKLOADS))
    ap.add_argument("--second-workload", default=SECOND,
                    help="measured the same way and reported under `workloads` ('' to skip)")
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--ring-groups", type=int, default=0,
                    help="ARNA hardware-aware ring with this many PE groups (8: one per die)")
    ap.add_argument("--cpu-budget", type=float, default=12.0,
                    help="seconds of oracle work at all threads (a third of it at one thread)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--grad-workload", default="arna_grad_512_256x4096",
                    choices=sorted(synth.WORKLOADS))
    ap.add_argument("--grad-frames", type=int, default=50,
                    help="frames of the fwd+bwd/fwd measurement (0: skip)")
    ap.add_argument("--batch-frames", type=int, default=20,
                    help="frames of the 64-sequence batched measurement (0: skip)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run 5 device-to-device copies of MIB MiB (counter calibration)")
    args = ap.parse_args()
    if args.calibrate_copy:
        import torch
        n = args.calibrate_copy * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes": 4 * n, "copies": 5}))
        return
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for {args.gpus}); the "
              "multi-GPU sharding of the path is a design note, not code", file=sys.stderr)
        sys.exit(2)

    def summary(g):
        c = g["cfg"]
        n = c["n_filters"] * c["n_pe"] * c["n_per_pe"]
        ms_step = g["total_ms"] / max(args.steps, 1)
        b_launch = algorithmic_bytes(n, c["width"], c["height"])
        k_ms = g["step_kernel_ms"]
        return dict(n=n, ms=ms_step, value=n * args.steps / (g["total_ms"] / 1e3),
                    plain_ms=g["plain_ms"] / max(args.steps, 1), bytes_launch=b_launch,
                    kernel_ms=k_ms, achieved=b_launch / (k_ms / 1e3) / 1e9)

    g = gpu_leg(args.workload, args.steps, args.warmup, args.seed, args.probe, args.ring_groups)
    cfg = g["cfg"]
    h = summary(g)
    N, ms, value = h["n"], h["ms"], h["value"]
    # the roofline of the step kernel: algorithmic bytes of one launch over its
    # average duration, from the events the library records around each step
    # launch on the kernels' stream (the timed region's per-step time also
    # holds the master-step launch and the gaps between launches)
    achieved = h["achieved"]
    counters = measured_counters(args.workload, args.ring_groups)
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
                   "ring_groups": cfg.get("ring_groups", 0),
                   "master_step": "every iteration, to a device trajectory (pf_run_traj)",
                   "parallelism": "one PE per workgroup, 1 GPU"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": (counters or {}).get("bytes_per_launch"),
                     "l2_hit_rate": (counters or {}).get("l2_hit_rate"),
                     "kernel": "k_step", "kernel_ms": h["kernel_ms"],
                     "bytes_per_launch": h["bytes_launch"], "kernel_sha": kernel_sha(),
                     "timed_region_ms_per_step": ms},
        "ms_per_step_without_master_record": h["plain_ms"],
        "valu": valu_entry(counters, h["kernel_ms"], N),
        "final_pe_eff": g["pe_eff"],
        "final_n_ex": g["n_ex"],
        "log_z_sum": g["log_z_sum"],
    }
    if args.second_workload:
        g2 = gpu_leg(args.second_workload, args.steps, args.warmup, args.seed, args.probe,
                     args.ring_groups)
        h2 = summary(g2)
        line["workloads"] = {
            w: {"value": x["value"], "ms_per_step": x["ms"],
                "ms_per_step_without_master_record": x["plain_ms"], "n_particles": x["n"],
                "kernel_ms": x["kernel_ms"], "roofline_frac": x["achieved"] / HBM_PEAK_GBS}
            for w, x in ((args.workload, h), (args.second_workload, h2))}
        if synth.WORKLOADS[args.second_workload]["filter"].get("init_mode") == 1:
            line["workloads"][args.second_workload]["phases"] = phase_leg(
                args.second_workload, args.seed)
    if args.grad_frames:
        gl = grad_leg(args.grad_workload, args.grad_frames, args.seed)
        line["fwd_bwd_over_fwd"] = gl["fwd_bwd_over_fwd"]
        line["grad"] = gl
    if args.batch_frames:
        from paper_1310_4624_amd.experiments import batch
        line["batch"] = batch(frames=args.batch_frames)
    if not args.no_cpu_baseline:
        cb = cpu_leg(args.workload, args.seed, args.cpu_budget, g["seq"])
        one = cpu_leg(args.workload, args.seed, args.cpu_budget / 3, g["seq"], threads=1)
        cb["cpu_model"] = cpu_model()
        cb["single_thread"] = {"value": one["value"], "cores": one["cores"], "sample": one["sample"]}
        line["cpu_baseline"] = cb
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
