"""Seeded synthetic video scenes for the global-illumination decomposition solver.

This module only *renders inputs*: it draws a scene (base colours, a Voronoi
reflectance map, a smooth direct-shading field and one Gaussian indirect blob per
base colour) and renders frames with the paper's image-formation model
(Sec. 4, eq. imageformation: I = R * sum_k b_k T_k with b_0 = white) plus i.i.d.
Gaussian noise.  It holds none of the solver's arithmetic (no energy, weights,
Jacobians or solves); both the FP64 oracle and the GPU library consume the
arrays it returns.

Scene recipe (stands in for the paper's real and SyntheticRoom videos, which
are not available):
  * base colours b_k ~ U[0.1, 0.9]^3, k = 1..K
  * m = max(8, K) Voronoi seeds s_i ~ U([0,W) x [0,H)), seed i carries colour
    perm(i) mod K; in video the seeds translate by (+1, 0) px per frame;
    the id of a pixel is the colour of the nearest seed to its centre
    (ties: lowest seed index); R is box-supersampled 2x2 unless point sampling
    is requested
  * direct shading D = 0.65 + 0.35 cos(2 pi (fx x/W + phx + 0.01 t)) cos(2 pi (fy y/H + phy)),
    fx, fy ~ U[0.5, 1.5], phx, phy ~ U[0, 1)  -> D in [0.3, 1.0]
  * indirect layer k: s_k = a_k exp(-|x - c_k(t)|^2 / (2 sigma_k^2)),
    a_k ~ U[0, A], sigma_k ~ U[0.05, 0.2] min(W, H), centre drifting 0.5 px/frame
  * I = R (D + sum_k s_k b_k) + N(0, noise^2) per channel, one noise stream per frame
    (spawned from the seed), so frames can be rendered in parallel
  * initial colour estimate b_init = clip(b + U[-0.05, 0.05]^3, 0.05, 0.95)
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class Clip:
    """A rendered clip.  Arrays are planar (channel-first) float32 unless noted."""

    width: int
    height: int
    K: int
    frames: np.ndarray          # (F, 3, H, W) float32, linear RGB
    ids: np.ndarray             # (F, H, W) uint8, colour index in [0, K)
    b_gt: np.ndarray            # (K, 3) float64, ground-truth base colours
    b_init: np.ndarray          # (K, 3) float64, perturbed initial estimate
    gt_r: np.ndarray            # (F, 3, H, W) float32, ln R
    gt_T: np.ndarray            # (F, K+1, H, W) float32, T_0 = D, T_k = s_k
    seed: int = 0
    meta: dict = field(default_factory=dict)

    @property
    def nframes(self) -> int:
        return int(self.frames.shape[0])


def _voronoi(px: np.ndarray, py: np.ndarray, sx: np.ndarray, sy: np.ndarray) -> np.ndarray:
    """Index of the nearest seed for each sample point; ties go to the lowest index."""
    best = np.full(px.shape, np.inf)
    arg = np.zeros(px.shape, dtype=np.int64)
    for i in range(sx.shape[0]):
        d = (px - sx[i]) ** 2 + (py - sy[i]) ** 2
        closer = d < best            # strict: an equal distance keeps the lower index
        best = np.where(closer, d, best)
        arg = np.where(closer, i, arg)
    return arg


def _scene(width, height, K, seed, amp, single_region):
    """Draw a scene's parameters from its seed (the scene stream of the seed)."""
    rng_scene = np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed).spawn(2)[0]))
    sc = {}
    sc["b"] = rng_scene.uniform(0.1, 0.9, size=(K, 3))
    m = max(8, K)
    sc["sx"] = rng_scene.uniform(0.0, width, size=m)
    sc["sy"] = rng_scene.uniform(0.0, height, size=m)
    sc["colour_of_seed"] = rng_scene.permutation(m) % K
    sc["fx"], sc["fy"] = rng_scene.uniform(0.5, 1.5, size=2)
    sc["phx"], sc["phy"] = rng_scene.uniform(0.0, 1.0, size=2)
    sc["a"] = rng_scene.uniform(0.0, amp, size=K)
    sc["sig"] = rng_scene.uniform(0.05, 0.2, size=K) * min(width, height)
    sc["cx0"] = rng_scene.uniform(0.0, width, size=K)
    sc["cy0"] = rng_scene.uniform(0.0, height, size=K)
    sc["theta"] = rng_scene.uniform(0.0, 2.0 * np.pi, size=K)
    sc["b_init"] = np.clip(sc["b"] + rng_scene.uniform(-0.05, 0.05, size=(K, 3)), 0.05, 0.95)
    if single_region:
        sc["colour_of_seed"][:] = 0
        sc["a"][:] = 0.0
    return sc


def _render(sc, width, height, K, t, supersample, single_region):
    """Noise-free frame t of a scene: (image, ids, R, T) in float64 / uint8."""
    b, cos_ = sc["b"], sc["colour_of_seed"]
    ys, xs = np.mgrid[0:height, 0:width].astype(np.float64)
    xc, yc = xs + 0.5, ys + 0.5
    stx = sc["sx"] + t
    vor_c = _voronoi(xc, yc, stx, sc["sy"])
    ids_t = cos_[vor_c]
    if supersample:
        R = np.zeros((3, height, width))
        offs = ((0.25, 0.25), (0.75, 0.25), (0.25, 0.75), (0.75, 0.75))
        for ox, oy in offs:
            R += b[cos_[_voronoi(xs + ox, ys + oy, stx, sc["sy"])]].transpose(2, 0, 1)
        R /= len(offs)
    else:
        R = b[ids_t].transpose(2, 0, 1)          # point sampling at the pixel centre
    if single_region:
        D = np.full((height, width), 0.65)
    else:
        D = 0.65 + 0.35 * np.cos(2 * np.pi * (sc["fx"] * xc / width + sc["phx"] + 0.01 * t)) * \
            np.cos(2 * np.pi * (sc["fy"] * yc / height + sc["phy"]))
    T = np.empty((K + 1, height, width))
    T[0] = D
    S = np.repeat(D[None], 3, axis=0)
    for k in range(K):
        ckx = sc["cx0"][k] + 0.5 * t * np.cos(sc["theta"][k])
        cky = sc["cy0"][k] + 0.5 * t * np.sin(sc["theta"][k])
        s_k = sc["a"][k] * np.exp(-((xc - ckx) ** 2 + (yc - cky) ** 2) / (2.0 * sc["sig"][k] ** 2))
        T[k + 1] = s_k
        S += s_k[None] * b[k][:, None, None]
    return R * S, ids_t, R, T


def _frame_noise(seed, t, shape, noise):
    """Noise of frame t: its own stream, spawned from the seed's noise stream, so
    frames can be rendered in any order."""
    seq = np.random.SeedSequence(seed).spawn(2)[1].spawn(t + 1)[t]
    return np.random.Generator(np.random.PCG64(seq)).normal(0.0, noise, size=shape)


def _render_into(out, sc, width, height, K, seed, t0, t1, supersample, noise, single_region, gt):
    frames, ids, gt_r, gt_T = out
    for t in range(t0, t1):
        img, ids_t, R, T = _render(sc, width, height, K, t, supersample, single_region)
        if noise > 0:
            img = img + _frame_noise(seed, t, img.shape, noise)
        frames[t] = img
        ids[t] = ids_t
        if gt:
            gt_r[t] = np.log(R)
            gt_T[t] = T


def make_clip(width: int, height: int, K: int, nframes: int, seed: int, *,
              amp: float = 0.2, supersample: bool = True, noise: float = 0.01,
              single_region: bool = False, gt: bool = True, workers: int = 1) -> Clip:
    """Render a seeded synthetic clip.

    single_region=True renders the degenerate scene used as an exact-recovery
    check: one colour everywhere, constant direct shading, no indirect light and
    no noise.  gt=False skips the ground-truth layers (gt_r, gt_T are None).
    workers > 1 renders frames in that many forked processes into shared
    memory; the result is the same as with one.
    """
    if width < 1 or height < 1 or K < 1 or nframes < 1:
        raise ValueError("bad clip shape")
    if single_region:
        noise = 0.0
    sc = _scene(width, height, K, seed, amp, single_region)
    F = nframes
    shapes = [((F, 3, height, width), np.float32), ((F, height, width), np.uint8)]
    if gt:
        shapes += [((F, 3, height, width), np.float32), ((F, K + 1, height, width), np.float32)]
    workers = max(1, min(int(workers), F))
    if workers == 1:
        out = [np.empty(sh, dt) for sh, dt in shapes]
    else:
        import mmap
        out = []
        for sh, dt in shapes:
            nbytes = int(np.prod(sh)) * np.dtype(dt).itemsize
            out.append(np.frombuffer(mmap.mmap(-1, max(1, nbytes)), dtype=dt, count=int(np.prod(sh))).reshape(sh))
    if not gt:
        out += [None, None]
    args = (sc, width, height, K, seed)
    if workers == 1:
        _render_into(out, *args, 0, F, supersample, noise, single_region, gt)
    else:
        import multiprocessing as mp
        ctx = mp.get_context("fork")
        bounds = [F * j // workers for j in range(workers + 1)]
        procs = [ctx.Process(target=_render_into,
                             args=(out, *args, bounds[j], bounds[j + 1], supersample, noise, single_region, gt))
                 for j in range(workers)]
        for p in procs:
            p.start()
        for p in procs:
            p.join()
        if any(p.exitcode != 0 for p in procs):
            raise RuntimeError("a frame-rendering worker failed")
        out = [None if o is None else np.array(o) for o in out]
    frames, ids, gt_r, gt_T = out
    return Clip(width, height, K, frames, ids, sc["b"], sc["b_init"], gt_r, gt_T, seed,
                meta=dict(amp=amp, supersample=supersample, noise=noise,
                          single_region=single_region))


def downsample_clip(clip: Clip, factor: int) -> Clip:
    """Area-average frames and ground truth over factor x factor blocks.

    Ids take the most frequent colour of each block (ties: lowest index).
    """
    F, _, H, W = clip.frames.shape
    h, w = H // factor, W // factor

    def area(x: np.ndarray) -> np.ndarray:
        x = x[..., : h * factor, : w * factor].astype(np.float64)
        return x.reshape(*x.shape[:-2], h, factor, w, factor).mean(axis=(-3, -1)).astype(np.float32)

    blocks = clip.ids[:, : h * factor, : w * factor].reshape(F, h, factor, w, factor)
    blocks = blocks.transpose(0, 1, 3, 2, 4).reshape(F, h, w, factor * factor).astype(np.int64)
    counts = np.zeros((F, h, w, clip.K), np.int64)
    for k in range(clip.K):
        counts[..., k] = (blocks == k).sum(axis=-1)
    ids = counts.argmax(axis=-1).astype(np.uint8)
    if clip.gt_r is None:
        gr = gT = None
    else:
        gr = np.log(area(np.exp(clip.gt_r.astype(np.float64)))).astype(np.float32)
        gT = area(clip.gt_T)
    return Clip(w, h, clip.K, area(clip.frames), ids, clip.b_gt.copy(), clip.b_init.copy(), gr, gT, clip.seed,
                meta=dict(clip.meta, downsampled_from=(W, H), factor=factor))


# --- named workloads -------------------------------------------------------

#: The solver schedule and problem shape of each named workload.
WORKLOADS = {
    "single_64x48_k4": dict(width=64, height=48, K=4, frames=1, seed=100, G=5, P=10,
                            temporal=False, amp=0.2, supersample=True),
    "video_640x480_k6": dict(width=640, height=480, K=6, frames=30, seed=200, G=3, P=8,
                             temporal=True, amp=0.2, supersample=True),
    "video_1280x720_k8": dict(width=1280, height=720, K=8, frames=60, seed=301, G=3, P=8,
                              temporal=True, amp=0.2, supersample=True),
    "video_1920x1080_k10": dict(width=1920, height=1080, K=10, frames=120, seed=500, G=3, P=8,
                                temporal=True, amp=0.35, supersample=False),
}

#: Clip sizes of the mixed batch of uneven clips.
MIXED_SIZES = ((320, 240), (640, 480), (960, 540), (1280, 720))


def workload_clip(name: str, nframes: int | None = None, **kw) -> Clip:
    w = WORKLOADS[name]
    return make_clip(w["width"], w["height"], w["K"], nframes or w["frames"], w["seed"],
                     amp=w["amp"], supersample=w["supersample"], **kw)


def mixed_batch_specs(nclips: int = 16, base_seed: int = 400):
    """Per-clip (width, height, frames, K, seed) of the mixed uneven batch."""
    out = []
    for j in range(nclips):
        rng = np.random.Generator(np.random.PCG64(base_seed + j))
        w, h = MIXED_SIZES[j % len(MIXED_SIZES)]
        frames = int(rng.integers(8, 33))
        K = int(rng.integers(4, 9))
        out.append(dict(width=w, height=h, frames=frames, K=K, seed=base_seed + j))
    return out
