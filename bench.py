#!/usr/bin/env python3
"""Decomposed Mpixel/s at a fixed final energy on one MI355X: the learned warm
start against the plain method.

Default workload: 1920x1080, 120 frames, K = 10, the plain schedule G x P = 3 x 8
(Sec. 7.1: G outer iterations of a layer step with P PCG iterations and a
base-colour step), temporal prior on.  Frame 0 (which has no previous frame to
warm-start from) is solved once with the plain schedule and checkpointed; a
step then decomposes frames 1..F-1 from that checkpoint.

  plain    every frame warm-started from the previous result, fixed 3 x 8.
  learned  the network's prediction from the previous result, judged against
           it by the energy, then outer iterations (P or fewer PCG iterations
           each: 8, 7, 6 and 5 are tried) until the frame's energy is at or below
           the plain method's final energy on that frame times (1 + 1e-4), up to
           twice the plain schedule's PCG iterations (device-side stop, no host
           trips).  Network inference, the judge and every energy evaluation
           are timed.  The same continuation from the plain start (no network)
           is reported as the control.

The learned run counts as matched when every frame meets its target.  `value`
is the throughput at the fixed final energy: the learned path's when matched
and faster, else the plain path's (config.method says which); both are
reported, with the speed-up.  Inputs are resident in device memory before
timing starts.

Also reported: the roofline of the dominant kernel (the PCG iteration, vector
updates fused with the matrix-free J^T J product; HIP events on the solver's
stream in a profiled pass) against the algorithmic bytes per pixel of the
method, (7n + 1 + tau) * 4 per PCG iteration, and per frame
4 G [P (7n + 1 + tau) + 7n + 7 + 3 tau]; the FP64 oracle timed on the host on a
bounded sample (one full-size frame) and on the 96 x 54 area-averaged copy of
the clip; plain-method lines for 640x480 and 1280x720; and the batch of 16
uneven clips (shared launches against one clip after another).
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
METRIC = "decomposed Mpixel/s at fixed final energy (1 GPU); learned warm-start vs plain"
GEN_WORKERS = 16


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def method_bytes(n: int, tau: int, G: int, P: int) -> dict:
    """Algorithmic bytes per pixel of the method (FP32 state, operator recomputed
    from the unknowns, q kept on chip): a PCG iteration reads u, the per-pixel
    data and the state and reads and writes x, r and p, (7n + 1 + tau) * 4; the
    build (3n + 4 + 3 tau) * 4, the apply 3n * 4, the base-colour sums (n + 3) * 4."""
    it = 7 * n + 1 + tau
    return dict(pcg=4 * it, frame=4 * G * (P * it + 7 * n + 7 + 3 * tau))


def impl_bytes(n: int, tau: int, P: int) -> float:
    """Bytes per pixel the implementation's PCG launches move on average: with
    the vectors carried in preconditioned form an iteration i > 1 reads u, z,
    M^-1 q, p and x (n planes each), the soft-Retinex weight and the temporal
    pair count, and writes x, z, p and M^-1 q (the Jacobi diagonal is rebuilt
    from u); iteration 1 starts x from zero; iteration 0 reads u and p0 and
    writes M^-1 q."""
    its = [3 * n + 1 + tau, 7 * n + 1 + tau] + [9 * n + 1 + tau] * max(0, P - 2)
    return 4.0 * sum(its[:P]) / max(P, 1)


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


def oracle_rate(clip, G, P, frames, what):
    """The FP64 oracle (test infrastructure, timed here only as the CPU baseline)
    on the first `frames` frames of a clip, one host thread."""
    from threadpoolctl import threadpool_limits
    import oracle as O
    with threadpool_limits(1):
        t0 = time.perf_counter()
        O.decompose_clip(clip.frames, clip.ids, clip.b_init, O.default_params(), G, P, temporal=True,
                         nframes=frames)
        dt = time.perf_counter() - t0
    px = frames * clip.width * clip.height
    return dict(value=px / dt / 1e6, unit="Mpx/s", cores=1, kind="oracle",
                sample=f"{what}: first {frames} frame(s) of {clip.width}x{clip.height} K={clip.K}, same "
                       f"{G}x{P} schedule, FP64 NumPy, 1 thread; {dt:.1f} s",
                host_cpus=os.cpu_count(), host_affinity=len(os.sched_getaffinity(0)))


class Video:
    """A clip resident on the device with a frame-0 checkpoint of the plain schedule."""

    def __init__(self, clip, G_, P_):
        import torch
        import paper_1908_01961_amd as G
        self.clip, self.G, self.P = clip, G_, P_
        self.K, self.W, self.H, self.F = clip.K, clip.width, clip.height, clip.nframes
        self.frames = torch.from_numpy(clip.frames).cuda()
        self.ids = torch.from_numpy(clip.ids).cuda()
        self.layers = torch.empty((self.K + 4, self.H, self.W), dtype=torch.float32, device="cuda")
        self.nb = 0
        s = self.solver()
        s.set_base_colors(clip.b_init)
        s.decompose_frame(self.frames[0], self.ids[0], self.layers)
        self.blob = s.save_state()
        # the launch shape from the library's autotuner, timed on the real layer
        # step of this frame (untimed here; every solver of the clip uses it)
        self.nb = s.autotune(None)
        s.close()
        self.px = (self.F - 1) * self.W * self.H

    def solver(self, G_=None, P_=None):
        import paper_1908_01961_amd as G
        s = G.Solver(self.W, self.H, G.default_params(self.K, gn_iters=G_ or self.G, pcg_iters=P_ or self.P,
                                                      temporal=1, refine_mode="every", record_energy=0,
                                                      use_graph=1))
        if self.nb:
            s.set_workgroups(self.nb)
        return s

    def pass_(self, s, targets=None, max_gn=0):
        """Frames 1..F-1 from the checkpoint; per-frame (energy, outer iterations)."""
        s.load_state(self.blob)
        return self.frames_(s, targets, max_gn)

    def frames_(self, s, targets=None, max_gn=0):
        """Frames 1..F-1 from the state the solver holds."""
        out = []
        for t in range(1, self.F):
            if targets is not None:
                s.set_energy_target(targets[t - 1], max_gn)
            _, st = s.decompose_frame(self.frames[t], self.ids[t], self.layers)
            out.append((st["energy_final"], st["gn_done"], st["warm_start_learned"]))
        return out

    def timed(self, s, steps, warmup, targets=None, max_gn=0):
        """Seconds per pass over frames 1..F-1.  Each pass starts from the frame-0
        checkpoint; restoring it (a host-to-device copy of the saved state, not part
        of any frame's work) happens before the pass's synchronised timed interval."""
        import torch
        for _ in range(warmup):
            self.pass_(s, targets, max_gn)
        total, last = 0.0, None
        for _ in range(steps):
            s.load_state(self.blob)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            last = self.frames_(s, targets, max_gn)
            torch.cuda.synchronize()
            total += time.perf_counter() - t0
        return total / steps, last


def kernel_roofline(video, s, workload):
    """Profiled pass (direct launches, HIP events around every launch on the
    solver's stream): the PCG iteration's average duration against the method's
    bytes, and each kernel's share."""
    s.set_profiling(True)
    video.pass_(s)
    kt = s.kernel_times()
    s.set_profiling(False)
    n, tau = video.K + 4, 1
    mv = kt["pcg"]
    avg_s = mv["ms"] / max(1, mv["launches"]) / 1e3
    npx = video.W * video.H
    mb = method_bytes(n, tau, video.G, video.P)["pcg"] * npx
    ib = impl_bytes(n, tau, video.P) * npx
    rf = dict(bound="hbm", kernel="k_pcg", achieved=round(mb / avg_s / 1e9, 1), peak=HBM_PEAK_GBS, unit="GB/s",
              frac=round(mb / avg_s / 1e9 / HBM_PEAK_GBS, 4), traffic=measured_traffic("k_pcg", workload),
              algorithmic_bytes_per_launch=mb, algorithmic_bytes_per_pixel=method_bytes(n, tau, video.G, video.P)["pcg"],
              avg_launch_us=round(avg_s * 1e6, 2),
              implementation_bytes_per_launch=round(ib), implementation_gbs=round(ib / avg_s / 1e9, 1))
    kernels = {k: dict(avg_us=round(v["ms"] * 1e3 / v["launches"], 2), launches=v["launches"],
                       share=round(v["ms"] / max(1e-12, sum(x["ms"] for x in kt.values())), 4))
               for k, v in kt.items() if v["launches"]}
    return rf, kernels


def frame_roofline(video, sec_per_frame):
    mb = method_bytes(video.K + 4, 1, video.G, video.P)["frame"] * video.W * video.H
    gbs = mb / sec_per_frame / 1e9
    return dict(achieved=round(gbs, 1), peak=HBM_PEAK_GBS, unit="GB/s", frac=round(gbs / HBM_PEAK_GBS, 4),
                algorithmic_bytes_per_frame=mb)


def train_network(video, train_frames, w):
    import paper_1908_01961_amd as G
    from paper_1908_01961_amd import warmstart as WSP
    W_, H_, K = video.W, video.H, video.K
    t0 = time.perf_counter()
    f = 2
    while (W_ // f) * (H_ // f) > 80000:
        f += 1
    tw, th = max(64, W_ // f), max(32, H_ // f)       # the workload's aspect, about 77k pixels
    # training scenes drawn from the workload's own recipe (indirect amplitude, edge sampling)
    store = WSP.make_training_set(K, tw, th, train_frames, 41, video.G, video.P, 10000, amp=w["amp"],
                                  supersample=w["supersample"])
    net_t = G.Net(K, tw, th)
    net_t.set_params(WSP.init_params(K, 1))
    hist = WSP.train(net_t, store, epochs=12, lr=4e-4)
    del store
    net = WSP.transfer(net_t, K, W_, H_)
    net_t.close()
    secs = time.perf_counter() - t0
    log(f"network trained on {train_frames} pairs at {tw}x{th} in {secs:.1f} s (loss {hist[-1]:.3e})")
    return net, dict(pairs=train_frames, size=f"{tw}x{th}", seconds=round(secs, 1), final_loss=hist[-1],
                     seeds="10000 and up")


def bench_video(args, clip, workload, learned=True):
    import numpy as np
    from scenes import WORKLOADS
    w = WORKLOADS[workload]
    video = Video(clip, w["G"], w["P"])
    s = video.solver()
    plain = video.pass_(s)
    E_plain = np.array([e for e, _, _ in plain])
    t_plain, _ = video.timed(s, args.steps, args.warmup)
    plain_mpx = video.px / t_plain / 1e6
    log(f"{workload} plain {w['G']}x{w['P']}: {t_plain * 1e3:.1f} ms per pass of {video.F - 1} frames, "
        f"{plain_mpx:.1f} Mpx/s")
    rf, kernels = kernel_roofline(video, s, workload)
    s.close()
    res = dict(video=video, t_plain=t_plain, plain_mpx=plain_mpx, roofline=rf, kernels=kernels,
               frame_roofline=frame_roofline(video, t_plain / (video.F - 1)), E_plain=E_plain)
    if not learned:
        return res
    net, train = train_network(video, args.train_frames, w)
    targets = E_plain * (1.0 + 1e-4)

    def run(Pl, with_net, steps, warmup):
        # at most twice the plain schedule's PCG iterations per frame; the energy is
        # checked from one outer iteration before the plain schedule's PCG budget
        # is spent (G P / Pl iterations), earlier checks being wasted on frames
        # that cannot have met the target yet
        max_gn = -(-2 * w["G"] * w["P"] // Pl)
        first_gn = max(1, (w["G"] * w["P"]) // Pl - 1)
        sl = video.solver(max_gn, Pl)
        sl.set_energy_check_from(first_gn)
        if with_net:
            sl.set_warmstart(net)
        t, last = video.timed(sl, steps, warmup, targets, max_gn)
        sl.close()
        E_l = np.array([e for e, _, _ in last])
        gn = np.array([g for _, g, _ in last])
        ex = E_l / E_plain - 1.0
        d = dict(pcg_iters=Pl, max_gn=max_gn, first_check=first_gn, mpx_s=round(video.px / t / 1e6, 2),
                 frames_s=round((video.F - 1) / t, 1), gn_mean=round(float(gn.mean()), 3), gn_max=int(gn.max()),
                 gn_histogram={int(g): int((gn == g).sum()) for g in np.unique(gn)},
                 energy_excess_max=float(ex.max()), energy_excess_median=float(np.median(ex)),
                 matched=bool(np.all(E_l <= targets)))
        if with_net:
            d["learned_start_taken"] = f"{int(sum(1 for _, _, k in last if k == 1))}/{video.F - 1}"
        return t, d

    # the continuation with the network's start and a reduced PCG count per outer
    # iteration (G x P is the plain method's reference schedule); the fastest
    # matched candidate is timed in full, and the same schedule from the plain
    # start (no network) is its control
    cands = []
    pcands = sorted({int(v) for v in args.learned_pcg.split(",")} if args.learned_pcg else {w["P"], 7, 6, 5},
                    reverse=True)
    for Pl in pcands:
        t, d = run(Pl, True, 2, 1)
        cands.append((t, d))
        log(f"learned, {Pl} PCG per outer iteration: {d}")
    ok = [(t, d) for t, d in cands if d["matched"]]
    best = min(ok, key=lambda td: td[0]) if ok else min(cands, key=lambda td: td[0])
    t_l, dl = run(best[1]["pcg_iters"], True, args.steps, args.warmup)
    t_c, dc = run(best[1]["pcg_iters"], False, 2, 1)
    net.close()
    matched = dl["matched"]
    log(f"learned + continuation: {t_l * 1e3:.1f} ms per pass, {dl['mpx_s']:.1f} Mpx/s, outer iterations "
        f"mean {dl['gn_mean']:.2f} (max {dl['gn_max']}), matched {matched}; plain start, same continuation: "
        f"{dc['mpx_s']:.1f} Mpx/s, matched {dc['matched']}")
    res["learned"] = dict(
        frames_timed=video.F - 1, criterion="E_learned[t] <= E_plain[t] * (1 + 1e-4) for every frame t >= 1",
        plain=dict(schedule=f"{w['G']}x{w['P']}", mpx_s=round(plain_mpx, 2),
                   frames_s=round((video.F - 1) / t_plain, 1)),
        learned=dl, candidates=[d for _, d in cands], control_plain_start_same_continuation=dc, train=train,
        speedup_at_matched_energy=round(t_plain / t_l, 3) if matched else None)
    res["t_learned"] = t_l
    return res


def bench_batch(args, clips):
    """Sixteen clips of mixed size (320x240 ... 1280x720), length (8-32 frames) and K
    (4-8), all advanced one frame per call through shared launches (gid_batch_*) in
    both launch layouts (every kernel one launch over all clips, or one launch per
    K; the figure is the layout the batch tuner keeps), against the same contexts
    solving the clips one after another.  Each clip's
    launch shape comes from the autotuner (untimed).  A pass covers every frame of
    every clip, from the initial colours."""
    import tempfile
    import torch
    import paper_1908_01961_amd as G
    solvers = [G.Solver(c.width, c.height, G.default_params(c.K, gn_iters=3, pcg_iters=8, temporal=1,
                                                            record_energy=0, use_graph=1)) for c in clips]
    frames = [torch.from_numpy(c.frames).cuda() for c in clips]
    ids = [torch.from_numpy(c.ids).cuda() for c in clips]
    shapes = []
    with tempfile.TemporaryDirectory() as d:
        for s, c, f, i in zip(solvers, clips, frames, ids):
            s.set_base_colors(c.b_init)
            s.load_frame(f[0], i[0])           # the tuner times the real layer step on a frame
            shapes.append(s.autotune(f"{d}/tune.txt"))
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

    def timed(fn, steps):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps

    steps = max(1, min(args.steps, 3))
    t_lay = {}
    for launch in ("one", "per_k"):          # both launch layouts of a batch step
        batch.set_launch(launch)
        t_lay[launch] = timed(step_batch, steps)
    chosen = batch.autotune()                # the library's choice (timed on the clips' last frames)
    t_b = t_lay[chosen]
    t_s = timed(step_sequential, steps)
    log(f"batch of {len(clips)}: one launch per kernel {px / t_lay['one'] / 1e6:.1f} Mpx/s, one launch per K "
        f"{px / t_lay['per_k'] / 1e6:.1f} Mpx/s (tuner: {chosen}), one clip after another {px / t_s / 1e6:.1f} Mpx/s")
    batch.close()
    for s in solvers:
        s.close()
    return dict(mpx_s=round(px / t_b / 1e6, 2), ms_per_pass=round(t_b * 1e3, 2), launch=chosen,
                one_launch_mpx_s=round(px / t_lay["one"] / 1e6, 2),
                per_k_mpx_s=round(px / t_lay["per_k"] / 1e6, 2),
                sequential_mpx_s=round(px / t_s / 1e6, 2), batched_over_sequential=round(t_s / t_b, 3),
                pixels_per_pass=px, clips=[dict(width=c.width, height=c.height, frames=c.nframes, K=c.K,
                                                workgroups=n) for c, n in zip(clips, shapes)])


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="video_1920x1080_k10")
    ap.add_argument("--frames", type=int, default=None, help="frames per clip (default: the workload's)")
    ap.add_argument("--learned", choices=("on", "off"), default="on")
    ap.add_argument("--train-frames", type=int, default=3000, help="training pairs for the learned warm start")
    ap.add_argument("--learned-pcg", default="",
                    help="PCG iterations per outer iteration tried with the learned start, comma-separated "
                         "(default: the workload's, 7, 6, 5)")
    ap.add_argument("--extras", choices=("on", "off", "batch"), default="on",
                    help="also the 640x480 and 1280x720 plain lines and the 16-clip batch (batch: the batch only)")
    ap.add_argument("--cpu", choices=("on", "off"), default="on", help="time the FP64 oracle on the host")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="after the run, copy a buffer of this many MiB device-to-device 5 times: a plain copy "
                         "of known size for scaling hardware byte counters (0: skip)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the solver runs on one GPU (independent clips would shard across "
              "GPUs with no communication); run with --gpus 1", file=sys.stderr)
        return 2

    # inputs are rendered on the host before anything touches the GPU (the renderer forks)
    from scenes import WORKLOADS, downsample_clip, make_clip, mixed_batch_specs, workload_clip
    w = WORKLOADS[args.workload]
    F = args.frames or w["frames"]
    t0 = time.perf_counter()
    clip = workload_clip(args.workload, nframes=F, gt=False, workers=GEN_WORKERS)
    log(f"generated {args.workload} ({F} frames) in {time.perf_counter() - t0:.1f} s")
    extra_clips = {}
    if args.extras != "off":
        for name in ("video_640x480_k6", "video_1280x720_k8"):
            if name != args.workload and args.extras == "on":
                extra_clips[name] = workload_clip(name, gt=False, workers=GEN_WORKERS)
        specs = mixed_batch_specs(16, 400)
        extra_clips["batch_16_mixed"] = [make_clip(sp["width"], sp["height"], sp["K"], sp["frames"], sp["seed"],
                                                   gt=False, workers=GEN_WORKERS) for sp in specs]
        log("generated the extra workloads")

    import torch
    torch.cuda.set_device(0)
    import paper_1908_01961_amd as G
    G.load_library()

    main_res = bench_video(args, clip, args.workload, learned=args.learned == "on")
    video = main_res["video"]
    lv = main_res.get("learned")
    use_learned = bool(lv and lv["learned"]["matched"] and main_res["t_learned"] < main_res["t_plain"])
    t_val = main_res["t_learned"] if use_learned else main_res["t_plain"]
    value = video.px / t_val / 1e6

    extras = {}
    for name, c in extra_clips.items():
        if name == "batch_16_mixed":
            extras[name] = bench_batch(args, c)
        else:
            r = bench_video(argparse.Namespace(steps=max(1, min(args.steps, 3)), warmup=1), c, name, learned=False)
            extras[name] = dict(mpx_s=round(r["plain_mpx"], 2), frames=c.nframes, roofline=r["roofline"],
                                frame_roofline=r["frame_roofline"])

    cpu = cpu96 = None
    if args.cpu == "on":
        log("oracle on one full-size frame")
        cpu = oracle_rate(clip, w["G"], w["P"], 1, "full-size sample")
        if args.workload == "video_1920x1080_k10":
            small = downsample_clip(clip, 20)
            cpu96 = oracle_rate(small, w["G"], w["P"], small.nframes, "the clip's 96x54 area-averaged copy")

    out = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "Mpx/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(t_val * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 (f64 reductions)",
        "data": "synthetic",
        "config": {"workload": args.workload, "width": video.W, "height": video.H, "frames": video.F, "K": video.K,
                   "frames_timed": video.F - 1, "gn_iters": video.G, "pcg_iters": video.P, "temporal": True,
                   "refine": "every", "graph": True, "workgroups": video.nb,
                   "method": "learned warm start + energy-target continuation" if use_learned else "plain"},
        "roofline": main_res["roofline"],
        "cpu_baseline": cpu,
        "cpu_baseline_96x54_copy": cpu96,
        "plain_mpx_s": round(main_res["plain_mpx"], 2),
        "learned_vs_plain": lv,
        "frame_roofline": main_res["frame_roofline"],
        "kernels": main_res["kernels"],
        "extras": extras,
    }
    print(json.dumps(out), flush=True)
    if args.calib_copy_mib > 0:
        nbytes = args.calib_copy_mib << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"calibration copy: 5 x {nbytes} bytes read and written")
    return 0


if __name__ == "__main__":
    sys.exit(main())
