"""The benchmark modes of Sec. V on the GPU path.

information sharing (Sec. V-B, Fig. 3): PE 0 starts at the object, every other
  PE uniformly over the state space; we count the iterations until every PE's
  estimate x^m is within a radius of the true position, and record the
  fraction of such PEs and PE_eff / M after every iteration.
  ``curves`` repeats it at the PE counts of Fig. 3 (24, 96, 192, 384).
tracking (Sec. V-A, Fig. 2): every PE starts at the true state; we record the
  RMSE of the master estimate against the truth and the exchange counts
  (Gaussian or Poisson pixel noise).
rmse40 (Fig. 2 right): tracking with 40 particles per PE over growing PE counts.
scaling (Fig. 2 left): a fixed total of 2^20 particles spread over more and
  more PEs; the GPU time per iteration of ARNA and RNA-0/10/50%.

Run as ``python -m paper_1310_4624_amd.experiments <what> [...]``; prints one
JSON object per run.
"""
from __future__ import annotations

import argparse
import json
import sys

import numpy as np

from . import synth
from .tracker import TRAJ_RECORD_BYTES, Tracker, trajectory

MODES = {"arna": (1, 0.1), "rna0": (0, 0.0), "rna10": (0, 0.1), "rna50": (0, 0.5)}


def _frames(seq):
    import torch
    return torch.from_numpy(seq.frames).cuda()


def infoshare(mode: str, seq_seed: int = 1000, filter_seed: int = 1, n_pe: int = 256,
              n_per_pe: int = 4096, steps: int = 200, radius: float = 2.0, seq=None,
              ring_groups: int = 0) -> dict:
    wl = "arna_infoshare_512_256x4096"
    mflag, ratio = MODES[mode]
    cfg = synth.filter_config(wl, mode=mflag, fixed_ratio=ratio, initial_ratio=0.1,
                              n_pe=n_pe, n_per_pe=n_per_pe, seed=filter_seed,
                              ring_groups=ring_groups)
    seq = seq if seq is not None else synth.make_sequence(wl, seed=seq_seed, frames=steps)
    frames = _frames(seq)
    tr = Tracker(cfg, seq.initial_truth()[:1])
    within, pe_eff, n_ex = [], [], []
    converged_at = None
    for k in range(1, min(steps, seq.frames.shape[0]) + 1):
        tr.step(frames[k - 1])
        est = tr.estimate()
        d = np.hypot(est["x_pe"][0, :, 0] - seq.truth[k, 0, 0],
                     est["x_pe"][0, :, 1] - seq.truth[k, 0, 1])
        frac = float(np.mean(d <= radius))
        within.append(frac)
        pe_eff.append(float(est["pe_eff"][0]) / n_pe)
        n_ex.append(int(est["n_ex"][0]))
        if converged_at is None and frac == 1.0:
            converged_at = k
    tr.close()
    return dict(mode=mode, n_pe=n_pe, n_per_pe=n_per_pe, seq_seed=seq_seed,
                ring_groups=ring_groups,
                filter_seed=filter_seed, steps=len(within), converged_at=converged_at,
                fraction_within=within, pe_eff_over_m=pe_eff, n_ex=n_ex)


def tracking(mode: str, seq_seed: int = 1000, filter_seed: int = 1, steps: int = 100,
             seq=None, workload: str = "arna_tracking_512_4x64x4096", q_true=None,
             **over) -> dict:
    wl = workload
    mflag, ratio = MODES[mode]
    cfg = synth.filter_config(wl, mode=mflag, fixed_ratio=ratio, seed=filter_seed, **over)
    seq = seq if seq is not None else synth.make_sequence(wl, seed=seq_seed, frames=steps,
                                                          q_true=q_true)
    import torch
    frames = _frames(seq)
    F = cfg["n_filters"]
    K = min(steps, seq.frames.shape[0])
    tr = Tracker(cfg, seq.initial_truth()[:F])
    # the master step of every iteration (Alg. 3 steps 9-10) to a device
    # trajectory, read back once: its rows are the stepwise estimates
    traj = torch.zeros(K * F * TRAJ_RECORD_BYTES, dtype=torch.uint8, device=frames.device)
    tr.run_traj(frames[:K], traj)
    rows = trajectory(traj, K, F)
    tr.close()
    err2 = np.sum((rows["xhat"][:, :, :2] - seq.truth[1:K + 1, :F, :2]) ** 2, axis=2)
    n_ex = rows["n_ex"]
    return dict(mode=mode, workload=wl, n_pe=cfg["n_pe"], n_per_pe=cfg["n_per_pe"],
                q_true=q_true if q_true is not None
                else synth.WORKLOADS[wl]["seq"].get("q_true", cfg["q"]),
                seq_seed=seq_seed, filter_seed=filter_seed, steps=len(err2),
                rmse_per_spot=np.sqrt(err2.mean(axis=0)).tolist(),
                rmse=float(np.sqrt(err2.mean())), mean_n_ex=np.mean(n_ex, axis=0).tolist())


def scaling(mode: str, n_pe: int, total: int = 1 << 20, steps: int = 30, warmup: int = 5,
            seq=None, tune: bool = False, **shape) -> dict:
    """GPU time per iteration with `total` particles over n_pe PEs (one spot,
    512^2, every particle starting at the truth); shape: block_size /
    pes_per_wg, or tune=True for the autotuner's choice."""
    import torch
    wl = "arna_grad_512_256x4096"
    mflag, ratio = MODES[mode]
    cfg = synth.filter_config(wl, mode=mflag, fixed_ratio=ratio, n_pe=n_pe,
                              n_per_pe=total // n_pe, **shape)
    seq = seq if seq is not None else synth.make_sequence(wl, seed=1000, frames=warmup + steps)
    frames = _frames(seq)
    if tune:
        from . import autotune
        cfg.update(autotune.tune(cfg, seq.initial_truth()[:1], frames, steps=6))
    tr = Tracker(cfg, seq.initial_truth()[:1])
    tr.run(frames[:warmup])
    torch.cuda.synchronize()
    ms = tr.run_timed(frames[warmup:warmup + steps]).astype(np.float64)
    est = tr.estimate()
    tr.close()
    ks = warmup + 1 + np.arange(steps)
    ring = (ks - 1) % 64 == 0 if mflag == 1 else np.zeros(steps, bool)
    return dict(mode=mode, n_pe=n_pe, n_per_pe=total // n_pe, total=total,
                block_size=cfg.get("block_size", 0), pes_per_wg=cfg.get("pes_per_wg", 0),
                us_per_step=float(ms[~ring].mean() * 1e3), n_ex=int(est["n_ex"][0]))


def batch(frames: int = 20, n_seq: int = 64, tune: bool = True, seed: int = 2000,
          call: int = 5) -> dict:
    """The batched workload: n_seq independent sequences of uneven size run
    (a) one after another, one launch per sequence and iteration, (b) as one
    batch (one launch per kernel variant and iteration), (c) the batch as HIP
    graphs, (d) (b) and (c) with the launch shapes (workgroup size, PEs per
    workgroup) chosen by the autotuner.
    Like a serving loop, (b) and (c) take the frames in calls of `call`
    iterations: the first call (untimed) loads the kernels and, in (c),
    captures the graph of a `call`-iteration run, which the timed calls
    replay.  Every mode times the same frames (all but the first `call`).
    Throughput = total particle-steps / time between two events."""
    import torch
    from . import autotune
    from .tracker import Batch
    seqs = synth.batch_sequences(seed=seed, n_seq=n_seq, frames=frames)
    dev = [torch.from_numpy(fr).cuda() for _, _, fr in seqs]
    timed_frames = frames - call
    total = sum(c["n_filters"] * c["n_pe"] * c["n_per_pe"] for c, _, _ in seqs) * timed_frames
    stream = torch.cuda.current_stream()

    def timed(fn):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1)

    def make(shapes=None):
        return [Tracker(dict(c, **(shapes[i] if shapes else {})), t)
                for i, (c, t, _) in enumerate(seqs)]

    def batched(shapes, graph):
        trs = make(shapes)
        b = Batch(trs)
        b.run([d[:call] for d in dev], graph=graph)
        ms = timed(lambda: [b.run([d[t0:t0 + call] for d in dev], graph=graph)
                            for t0 in range(call, frames, call)])
        x = [t.estimate()["x_global"] for t in trs]
        b.close()
        for t in trs:
            t.close()
        return ms, x

    out = {"n_seq": n_seq, "frames": frames, "frames_per_call": call,
           "timed_frames": timed_frames, "particle_steps": total}
    # warm-up: load every kernel variant once, per context (two iterations,
    # so that multi-iteration launches are loaded too)
    trs = make()
    for t, d in zip(trs, dev):
        t.run(d[:2])
    for t in trs:
        t.close()
    trs = make()
    for t, d in zip(trs, dev):
        t.run(d[:call])
    ms = timed(lambda: [t.run(d[call:]) for t, d in zip(trs, dev)])
    ref = [t.estimate()["x_global"] for t in trs]
    for t in trs:
        t.close()
    out["sequential_ms"] = ms
    for name, graph in (("batched_ms", False), ("batched_graph_ms", True)):
        ms, x = batched(None, graph)
        out[name] = ms
        out[name.replace("_ms", "_equal")] = all(np.array_equal(a, r) for a, r in zip(x, ref))
    if tune:
        shapes = [autotune.tune(c, t, d, steps=min(6, frames - 2)) for (c, t, _), d in zip(seqs, dev)]
        for name, graph in (("batched_tuned_ms", False), ("batched_graph_tuned_ms", True)):
            out[name], _ = batched(shapes, graph)
        out["tuned_shapes"] = [[s["block_size"], s["pes_per_wg"]] for s in shapes]
        out["default_block_sizes"] = [min(1024, (c["n_per_pe"] + 63) // 64 * 64) for c, _, _ in seqs]
    for k in list(out):
        if k.endswith("_ms"):
            out[k.replace("_ms", "_particle_steps_per_s")] = total / (out[k] / 1e3)
    return out


def infoshare_study(seeds: int = 10, modes=("arna", "rna0", "rna10", "rna50"),
                    n_pe: int = 256, n_per_pe: int = 4096, steps: int = 200,
                    curve_pes=(24, 96, 192, 384), curve_steps: int = 20,
                    curve_n_per_pe: int = 4096) -> dict:
    """The information-sharing result of Sec. V-B / Fig. 3 over several seeds:
    per mode the iterations until every PE estimate is within 2 px of the spot
    (None: not within `steps`; the median counts those as later than any
    converged run), and PE_eff / M after 10 and 20 iterations at the PE counts
    of Fig. 3.  Seed s uses sequence 1000 + s and filter seed 1 + s for every
    mode, so the modes see the same frames and start."""
    runs = {m: [] for m in modes}
    for s in range(seeds):
        # the workload's full sequence (200 frames) whatever `steps` is: its
        # frames do not depend on how many iterations are run
        seq = synth.make_sequence("arna_infoshare_512_256x4096", seed=1000 + s)
        for m in modes:
            r = infoshare(m, seq_seed=1000 + s, filter_seed=1 + s, n_pe=n_pe, n_per_pe=n_per_pe,
                          steps=steps, seq=seq)
            print(f"infoshare seed {s} {m}: converged at {r['converged_at']}", file=sys.stderr,
                  flush=True)
            runs[m].append(dict(seed=s, converged_at=r["converged_at"],
                                within_at_10=r["fraction_within"][9],
                                within_at_20=r["fraction_within"][19],
                                pe_eff_over_m_at_10=r["pe_eff_over_m"][9],
                                pe_eff_over_m_at_20=r["pe_eff_over_m"][19]))

    def median_steps(rs):
        v = sorted(steps + 1 if r["converged_at"] is None else r["converged_at"] for r in rs)
        med = float(np.median(v))
        return None if med > steps else med

    summary = {m: dict(median_converged_at=median_steps(rs),
                       converged_runs=sum(r["converged_at"] is not None for r in rs),
                       runs=len(rs)) for m, rs in runs.items()}
    curves = {}
    cseqs = [synth.make_sequence("arna_infoshare_512_256x4096", seed=1000 + s, frames=curve_steps)
             for s in range(seeds)]
    for n in curve_pes:
        for m in modes:
            vals = {10: [], 20: []}
            for s in range(seeds):
                seq = cseqs[s]
                r = infoshare(m, seq_seed=1000 + s, filter_seed=1 + s, n_pe=n, n_per_pe=curve_n_per_pe,
                              steps=curve_steps, seq=seq)
                for i in vals:
                    if i <= len(r["pe_eff_over_m"]):
                        vals[i].append(r["pe_eff_over_m"][i - 1])
            print(f"PE_eff curves {n} PEs {m} done", file=sys.stderr, flush=True)
            curves.setdefault(str(n), {})[m] = {
                f"pe_eff_over_m_at_{i}": dict(median=float(np.median(v)), min=float(min(v)),
                                              max=float(max(v)))
                for i, v in vals.items() if v}
    return dict(experiment="information sharing (Sec. V-B, Fig. 3)", n_pe=n_pe,
                n_per_pe=n_per_pe, steps=steps, radius_px=2.0, seeds=seeds, summary=summary,
                runs=runs, pe_eff_curves=dict(n_per_pe=curve_n_per_pe, steps=curve_steps,
                                              by_pe_count=curves))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("what", choices=["infoshare", "curves", "tracking", "rmse40", "scaling",
                                     "batch", "infoshare-study"])
    ap.add_argument("--out", default="",
                    help="infoshare-study, rmse40, scaling, tracking: also write the results (with the "
                         "command line) as JSON here")
    ap.add_argument("--workload", default="arna_tracking_512_4x64x4096")
    ap.add_argument("--ring-groups", type=int, default=0)
    ap.add_argument("--modes", default="arna,rna10,rna50,rna0")
    ap.add_argument("--seeds", type=int, default=1)
    ap.add_argument("--n-pe", type=int, default=256)
    ap.add_argument("--n-per-pe", type=int, default=4096)
    ap.add_argument("--steps", type=int, default=0)
    ap.add_argument("--curves", action="store_true", help="include the per-step curves")
    ap.add_argument("--shapes", default="",
                    help="scaling: only these PE counts and launch shapes, as n_pe:BxP,... "
                         "(B = block_size, P = pes_per_wg; 0x0 = the defaults)")
    ap.add_argument("--q-true", type=float, default=None,
                    help="tracking: process noise of the true trajectories (default: the "
                         "workload's)")
    ap.add_argument("--tuned", action="store_true",
                    help="scaling: also the autotuner's launch shape (workgroup size, PEs per "
                         "workgroup)")
    args = ap.parse_args()
    out = []
    command = "python -m paper_1310_4624_amd.experiments " + " ".join(sys.argv[1:])

    def emit(r):
        out.append(r)
        print(json.dumps(r), flush=True)

    def store():
        if args.out:
            with open(args.out, "w") as fh:
                fh.write(json.dumps({"command": command, "records": out}, indent=1) + "\n")
    if args.what == "infoshare-study":
        r = infoshare_study(seeds=args.seeds, modes=tuple(args.modes.split(",")),
                            n_pe=args.n_pe, n_per_pe=args.n_per_pe, steps=args.steps or 200)
        r["command"] = "python -m paper_1310_4624_amd.experiments " + " ".join(sys.argv[1:])
        text = json.dumps(r, indent=1)
        if args.out:
            with open(args.out, "w") as fh:
                fh.write(text + "\n")
        print(json.dumps(r["summary"]), flush=True)
        return
    if args.what == "batch":
        print(json.dumps(batch(frames=args.steps or 20)), flush=True)
        return
    if args.what == "curves":
        for n_pe in (24, 96, 192, 384):
            for s in range(args.seeds):
                for mode in args.modes.split(","):
                    r = infoshare(mode, seq_seed=1000 + s, filter_seed=1 + s, n_pe=n_pe,
                                  n_per_pe=args.n_per_pe, steps=args.steps or 40,
                                  ring_groups=args.ring_groups)
                    r["pe_eff_over_m_at"] = {str(i): r["pe_eff_over_m"][i - 1]
                                             for i in (1, 2, 5, 10, 20, 40)
                                             if i <= len(r["pe_eff_over_m"])}
                    r["fraction_within_at"] = {str(i): r["fraction_within"][i - 1]
                                               for i in (1, 2, 5, 10, 20, 40)
                                               if i <= len(r["fraction_within"])}
                    if not args.curves:
                        for k in ("fraction_within", "pe_eff_over_m", "n_ex"):
                            r.pop(k)
                    print(json.dumps(r), flush=True)
        return
    if args.what == "rmse40":
        for n_pe in (24, 96, 384, 1536, 6144):
            for s in range(args.seeds):
                for mode in args.modes.split(","):
                    emit(tracking(mode, seq_seed=1000 + s, filter_seed=1 + s,
                                  steps=args.steps or 50, n_pe=n_pe, n_per_pe=40))
        store()
        return
    if args.what == "scaling":
        if args.shapes:   # "n_pe:BxP,...": given launch shapes only
            for item in args.shapes.split(","):
                n_pe, shape = item.split(":")
                bs, ppw = shape.split("x")
                for mode in args.modes.split(","):
                    emit(scaling(mode, int(n_pe), block_size=int(bs), pes_per_wg=int(ppw)))
            store()
            return
        for n_pe in (256, 512, 1024, 2048, 4096, 8192):
            for mode in args.modes.split(","):
                emit(dict(scaling(mode, n_pe), shape="default"))
                if args.tuned:
                    emit(dict(scaling(mode, n_pe, tune=True), shape="tuned"))
        store()
        return
    for s in range(args.seeds):
        for mode in args.modes.split(","):
            if args.what == "infoshare":
                r = infoshare(mode, seq_seed=1000 + s, filter_seed=1 + s, n_pe=args.n_pe,
                              n_per_pe=args.n_per_pe, steps=args.steps or 200,
                              ring_groups=args.ring_groups)
                if not args.curves:
                    r = {k: v for k, v in r.items()
                         if k not in ("fraction_within", "pe_eff_over_m", "n_ex")} | {
                        "fraction_within_at": {str(i): r["fraction_within"][i - 1]
                                               for i in (5, 10, 20, 50, 100, 200)
                                               if i <= len(r["fraction_within"])}}
            else:
                r = tracking(mode, seq_seed=1000 + s, filter_seed=1 + s,
                             steps=args.steps or 100, workload=args.workload,
                             q_true=args.q_true)
            emit(r)
    if args.what == "tracking":
        store()


if __name__ == "__main__":
    main()
