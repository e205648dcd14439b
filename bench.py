#!/usr/bin/env python3
"""Decomposed Mpixel/s of the alternating Gauss-Newton decomposition on one MI355X.

A step decomposes one whole synthetic clip: every frame goes through the fixed
schedule (G outer iterations of a layer step with P PCG iterations and a
base-colour step), warm-started from the previous frame with the temporal
prior on, starting from the initial colour estimate.  Inputs are resident in
device memory before timing starts; per-frame layers are written to device
memory.  Default workload: 640x480, 30 frames, K = 6, G x P = 3 x 8.

Prints one JSON line.  Besides the throughput it reports the roofline of the
dominant kernel (the PCG iteration: vector updates fused with the matrix-free
J^T J product, timed with HIP events on the solver's stream in a profiled pass
over the same clip) and the FP64 oracle
timed on host cores on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def algorithmic_bytes(n: int, tau: int, G: int, P: int) -> dict:
    """Bytes per pixel the method must move with FP32 state and the operator
    recomputed from the unknowns; the PCG vectors are carried in preconditioned
    form (z = M^-1 r and M^-1 q).  A PCG iteration i > 1 reads u, z, M^-1 q, p, x
    and M^-1 (n planes each), the soft-Retinex weight and the temporal pair count,
    and writes x, z, p and M^-1 q; iteration 1 starts x from zero and reads p0 = z0
    once; the first iteration reads u, p0 and M^-1 and writes M^-1 q.  The build
    reads u, the frame, the weight and the temporal sums and writes M^-1 and p0;
    the apply reads u, x and p and writes u."""
    its = [4 * n + 1 + tau, 8 * n + 1 + tau] + [10 * n + 1 + tau] * max(0, P - 2)
    pcg_total = sum(its[:P])
    build = 3 * n + 4 + 4 * tau
    apply = 4 * n + 3
    return dict(pcg=4 * pcg_total / max(P, 1),            # average per PCG launch
                frame=4 * G * (pcg_total + build + apply))


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch of a kernel from the committed rocprofv3 counter
    summary of this workload, or None when there is none or the kernel source
    has changed since the counters were taken."""
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}.md")
    src = os.path.join(ROOT, "paper_1908_01961_amd", "csrc", "gid_kernels.hip")
    try:
        text = open(path).read()
        h = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    except OSError:
        return None
    m = re.search(r"kernel=(\S+) traffic_bytes_per_launch=(\d+) kernel_source_sha256_16=([0-9a-f]+)", text)
    if not m or m.group(1) != kernel or m.group(3) != h:
        return None
    return int(m.group(2))


def cpu_baseline(clip, G, P, frames):
    from threadpoolctl import threadpool_limits
    import oracle as O
    with threadpool_limits(1):
        t0 = time.perf_counter()
        O.decompose_clip(clip.frames, clip.ids, clip.b_init, O.default_params(), G, P, temporal=True,
                         nframes=frames)
        dt = time.perf_counter() - t0
    px = frames * clip.width * clip.height
    return dict(value=px / dt / 1e6, unit="Mpx/s", cores=1, kind="oracle",
                sample=f"first {frames} frame(s) of the {clip.width}x{clip.height} K={clip.K} clip, "
                       f"same {G}x{P} schedule, FP64 NumPy, 1 thread; {dt:.1f} s",
                host_cpus=os.cpu_count(), host_affinity=len(os.sched_getaffinity(0)))


def learned_vs_plain(clip, w, train_frames: int, log):
    """The learned warm start against the plain method on the same clip.

    Frame 0 (no previous frame to warm-start from) runs the plain schedule and
    is checkpointed; every candidate then solves frames 1..F-1 from that
    checkpoint.  The network is trained first (untimed) on train_frames pairs
    from plain decompositions of synthetic clips with seeds disjoint from the
    workload's.  A schedule counts as matched when on every frame its final
    energy is at most the plain method's times (1 + 1e-4).  Timed passes run
    the frames back to back on the device; energies come from a separate pass
    with per-frame statistics."""
    import numpy as np
    import torch

    import paper_1908_01961_amd as G
    from paper_1908_01961_amd import warmstart as WSP

    W_, H_, K, F = clip.width, clip.height, clip.K, clip.nframes
    Gp, Pp = w["G"], w["P"]
    frames = torch.from_numpy(clip.frames).cuda()
    ids = torch.from_numpy(clip.ids).cuda()

    def ctx(g, p):
        return G.Solver(W_, H_, G.default_params(K, gn_iters=g, pcg_iters=p, temporal=1, refine_mode="every",
                                                 record_energy=0, use_graph=1))

    s0 = ctx(Gp, Pp)
    s0.set_base_colors(clip.b_init)
    s0.decompose_frame(frames[0], ids[0])
    blob = s0.save_state()
    s0.close()

    def run(g, p, net=None):
        s = ctx(g, p)
        s.load_state(blob)
        if net is not None:
            s.set_warmstart(net)
        E, taken = [], 0
        for t in range(1, F):
            _, st = s.decompose_frame(frames[t], ids[t])
            E.append(st["energy_final"])
            taken += st["warm_start_learned"] == 1
        best = None
        for _ in range(3):
            s.load_state(blob)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for t in range(1, F):
                s.decompose_frame_async(frames[t], ids[t])
            s.synchronize()
            dt = time.perf_counter() - t0
            best = dt if best is None else min(best, dt)
        s.close()
        return np.array(E), best, taken

    px = (F - 1) * W_ * H_
    E_plain, t_plain, _ = run(Gp, Pp)
    log(f"plain {Gp}x{Pp}: {px / t_plain / 1e6:.1f} Mpx/s on frames 1..{F - 1}")
    t0 = time.perf_counter()
    f = 2
    while (W_ // f) * (H_ // f) > 80000:
        f += 1
    tw, th = max(64, W_ // f), max(32, H_ // f)       # training frames: the workload's aspect, ~77k pixels
    store = WSP.make_training_set(K, tw, th, train_frames, 41, Gp, Pp, 10000)
    net_t = G.Net(K, tw, th)
    net_t.set_params(WSP.init_params(K, 1))
    hist = WSP.train(net_t, store, epochs=4, lr=1e-3)
    del store
    net = WSP.transfer(net_t, K, W_, H_)
    net_t.close()
    train_s = time.perf_counter() - t0
    log(f"network trained on {train_frames} pairs at {tw}x{th} in {train_s:.1f} s (loss {hist[-1]:.3e})")

    def summary(E, dt, taken=None):
        ex = E / E_plain - 1.0
        d = dict(mpx_s=round(px / dt / 1e6, 2), frames_s=round((F - 1) / dt, 1),
                 energy_excess_max=float(ex.max()), energy_excess_median=float(np.median(ex)),
                 matched=bool(ex.max() <= 1e-4))
        if taken is not None:
            d["learned_start_taken"] = f"{taken}/{F - 1}"
        return d

    scheds = []
    for g, p in ((1, Pp), (2, Pp), (Gp, Pp)):
        E_l, t_l, taken = run(g, p, net)
        row = dict(schedule=f"{g}x{p}", learned=summary(E_l, t_l, taken))
        if (g, p) != (Gp, Pp):
            E_r, t_r, _ = run(g, p)
            row["plain_same_schedule"] = summary(E_r, t_r)
        scheds.append(row)
        log(f"learned {g}x{p}: {row['learned']}")
    net.close()
    plain_mpx = px / t_plain / 1e6
    matched = [r for r in scheds if r["learned"]["matched"]]
    best = max(matched, key=lambda r: r["learned"]["mpx_s"]) if matched else None
    return dict(frames_timed=F - 1, plain=dict(schedule=f"{Gp}x{Pp}", mpx_s=round(plain_mpx, 2)),
                train=dict(pairs=train_frames, size=f"{tw}x{th}", seconds=round(train_s, 1), final_loss=hist[-1],
                           seeds="10000 and up"),
                schedules=scheds,
                criterion="E_learned[t] <= E_plain[t] * (1 + 1e-4) for every frame t >= 1",
                best_matched_schedule=best["schedule"] if best else None,
                speedup_at_matched_energy=round(best["learned"]["mpx_s"] / plain_mpx, 3) if best else None)


def bench_batch(args, log):
    """Sixteen clips of mixed size (320x240 ... 1280x720), length (8-32 frames) and K
    (4-8), all advanced one frame per call through shared launches (gid_batch_*),
    against the same contexts solving the clips one after another.  Each clip's
    launch shape comes from the autotuner (untimed).  A step is one pass over
    every frame of every clip, from the initial colours."""
    import tempfile

    import torch

    import paper_1908_01961_amd as G
    from scenes import make_clip, mixed_batch_specs

    specs = mixed_batch_specs(16, 400)
    clips = [make_clip(sp["width"], sp["height"], sp["K"], sp["frames"], sp["seed"]) for sp in specs]
    log(f"{len(clips)} clips generated")
    solvers = [G.Solver(c.width, c.height, G.default_params(c.K, gn_iters=3, pcg_iters=8, temporal=1,
                                                            record_energy=0, use_graph=1)) for c in clips]
    with tempfile.TemporaryDirectory() as d:
        shapes = [s.autotune(f"{d}/tune.txt") for s in solvers]
    frames = [torch.from_numpy(c.frames).cuda() for c in clips]
    ids = [torch.from_numpy(c.ids).cuda() for c in clips]
    Fmax = max(c.nframes for c in clips)
    px = sum(c.nframes * c.width * c.height for c in clips)
    batch = G.Batch(solvers)

    def step_batch():
        for s, c in zip(solvers, clips):
            s.set_base_colors(c.b_init)
        for t in range(Fmax):
            batch.step_async([frames[i][t] if t < c.nframes else None for i, c in enumerate(clips)],
                             [ids[i][t] if t < c.nframes else None for i, c in enumerate(clips)])
            batch.synchronize()

    def step_sequential():
        for i, (s, c) in enumerate(zip(solvers, clips)):
            s.set_base_colors(c.b_init)
            for t in range(c.nframes):
                s.decompose_frame_async(frames[i][t], ids[i][t])
            s.synchronize()

    def timed(fn):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / args.steps

    t_b = timed(step_batch)
    log(f"batched: {t_b * 1e3:.1f} ms per pass, {px / t_b / 1e6:.1f} Mpx/s")
    t_s = timed(step_sequential)
    log(f"one clip after another: {t_s * 1e3:.1f} ms per pass, {px / t_s / 1e6:.1f} Mpx/s")
    batch.close()
    for s in solvers:
        s.close()
    out = {
        "metric": "decomposed Mpixel/s at fixed final energy (1 GPU); learned warm-start vs plain",
        "value": round(px / t_b / 1e6, 2), "unit": "Mpx/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(t_b * 1e3, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32 (f64 reductions)", "data": "synthetic",
        "config": {"workload": "batch_16_mixed", "clips": [dict(width=c.width, height=c.height, frames=c.nframes,
                                                                K=c.K, workgroups=n) for c, n in zip(clips, shapes)],
                   "pixels_per_step": px, "gn_iters": 3, "pcg_iters": 8, "temporal": True, "method": "plain"},
        "sequential": {"mpx_s": round(px / t_s / 1e6, 2), "ms_per_step": round(t_s * 1e3, 3)},
        "batched_over_sequential": round(t_s / t_b, 3),
    }
    print(json.dumps(out), flush=True)
    return 0


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="video_640x480_k6")
    ap.add_argument("--frames", type=int, default=None, help="frames per clip (default: the workload's)")
    ap.add_argument("--no-graph", action="store_true", help="launch kernels directly instead of graph replay")
    ap.add_argument("--cpu-frames", type=int, default=8,
                    help="oracle sample size in frames, about 10 s of host work at 640x480 (0: skip)")
    ap.add_argument("--learned", choices=("on", "off"), default="on",
                    help="also compare the learned warm start with the plain method on the workload")
    ap.add_argument("--train-frames", type=int, default=2000, help="training pairs for the learned warm start")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="after the run, copy a buffer of this many MiB device-to-device 5 times: a plain copy "
                         "of known size for scaling hardware byte counters (0: skip)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the solver is single-GPU (clips would shard across GPUs with "
              "no communication); run with --gpus 1", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import paper_1908_01961_amd as G
    from scenes import WORKLOADS, workload_clip

    if args.workload == "batch_16_mixed":
        return bench_batch(args, lambda m: print(f"[bench] {m}", file=sys.stderr, flush=True))
    w = WORKLOADS[args.workload]
    F = args.frames or w["frames"]
    print(f"[bench] generating {args.workload} ({F} frames)", file=sys.stderr, flush=True)
    clip = workload_clip(args.workload, nframes=F)
    W_, H_, K = clip.width, clip.height, clip.K
    n = K + 4
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    frames = torch.from_numpy(clip.frames).to(dev)
    ids = torch.from_numpy(clip.ids).to(dev)
    layers = torch.empty((F, n, H_, W_), dtype=torch.float32, device=dev)
    prm = G.default_params(K, gn_iters=w["G"], pcg_iters=w["P"], temporal=int(w["temporal"]),
                           refine_mode="every", record_energy=0, use_graph=0 if args.no_graph else 1)
    solver = G.Solver(W_, H_, prm)

    def step():
        solver.set_base_colors(clip.b_init)
        for t in range(F):
            solver.decompose_frame_async(frames[t], ids[t], layers[t])
        return solver.synchronize()

    for i in range(args.warmup):
        step()
        print(f"[bench] warmup {i + 1}/{args.warmup} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record()
    last = None
    for _ in range(args.steps):
        last = step()
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)
    ms_per_step = wall * 1e3 / args.steps
    px = F * W_ * H_
    value = px * args.steps / wall / 1e6
    print(f"[bench] timed {args.steps} steps: {ms_per_step:.2f} ms/step, {value:.1f} Mpx/s", file=sys.stderr,
          flush=True)
    b_final, stats = last

    # profiled pass: per-kernel durations from HIP events on the solver's stream
    solver.set_profiling(True)
    step()
    kt = solver.kernel_times()
    solver.set_profiling(False)
    mv = kt["pcg"]
    mv_avg_s = mv["ms"] / max(1, mv["launches"]) / 1e3
    tau = 1 if w["temporal"] else 0
    ab = algorithmic_bytes(n, tau, w["G"], w["P"])
    mv_bytes = ab["pcg"] * W_ * H_
    achieved = mv_bytes / mv_avg_s / 1e9
    frame_ms = ms_per_step / F
    frame_gbs = ab["frame"] * W_ * H_ / (frame_ms / 1e3) / 1e9
    roofline = dict(bound="hbm", kernel="k_pcg", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(achieved / HBM_PEAK_GBS, 4), traffic=measured_traffic("k_pcg", args.workload),
                    algorithmic_bytes_per_launch=mv_bytes, avg_launch_us=round(mv_avg_s * 1e6, 2))
    kernels = {k: dict(avg_us=round(v["ms"] * 1e3 / v["launches"], 2), launches=v["launches"],
                       share=round(v["ms"] / max(1e-12, sum(x["ms"] for x in kt.values())), 4))
               for k, v in kt.items() if v["launches"]}

    learned = None
    if args.learned == "on":
        learned = learned_vs_plain(clip, w, args.train_frames,
                                   lambda m: print(f"[bench] {m}", file=sys.stderr, flush=True))

    cpu = None
    if args.cpu_frames > 0:
        print(f"[bench] oracle on {args.cpu_frames} frame(s)", file=sys.stderr, flush=True)
        cpu = cpu_baseline(clip, w["G"], w["P"], min(args.cpu_frames, F))

    out = {
        "metric": "decomposed Mpixel/s at fixed final energy (1 GPU); learned warm-start vs plain",
        "value": round(value, 2),
        "unit": "Mpx/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 (f64 reductions)",
        "data": "synthetic",
        "config": {"workload": args.workload, "width": W_, "height": H_, "frames": F, "K": K,
                   "gn_iters": w["G"], "pcg_iters": w["P"], "temporal": bool(w["temporal"]),
                   "refine": "every", "method": "plain", "graph": not args.no_graph},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "learned_vs_plain": learned,
        "frame_roofline": dict(achieved=round(frame_gbs, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                               frac=round(frame_gbs / HBM_PEAK_GBS, 4),
                               algorithmic_bytes_per_frame=ab["frame"] * W_ * H_),
        "gpu_event_ms_per_step": round(gpu_ms / args.steps, 3),
        "final_energy_last_frame": stats["energy_final"],
        "kernels": kernels,
    }
    print(json.dumps(out), flush=True)
    solver.close()
    if args.calib_copy_mib > 0:
        nbytes = args.calib_copy_mib << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(f"[bench] calibration copy: 5 x {nbytes} bytes read and written", file=sys.stderr, flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
