"""Training and use of the learned warm start (library calls only).

The network (include/gid.h, gid_net_*) learns the solver's own frame-to-frame
update: from the frame I_t and the previous result u_{t-1} it predicts
du = u_t - u_{t-1} and db = b_t - b_{t-1}, where (u_t, b_t) is what the plain
schedule produces for frame t from (u_{t-1}, b_{t-1}).  Training pairs come
from decomposing seeded synthetic clips with the GPU solver; the network is
trained on the GPU by its own forward, backward and Adam kernels.  The network
is fully convolutional with a global-average colour head, so weights trained at
one frame size serve any other (copied into a network created for that size).
"""
from __future__ import annotations

import time

import numpy as np

from .gid import Net, Solver, default_params

C_HID = 32
N_CONV = 6


def layer_shapes(K: int):
    """(c_in, c_out) of the six conv layers for K base colours."""
    n = K + 4
    return [(3 + n, C_HID)] + [(C_HID, C_HID)] * 4 + [(C_HID, n)]


def init_params(K: int, seed: int) -> np.ndarray:
    """He-normal conv weights and zero biases, with the output layer and the
    colour head at zero so the untrained network predicts no change (the judge
    then keeps the previous frame).  Layout of include/gid.h."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for l, (ci, co) in enumerate(layer_shapes(K)):
        if l < N_CONV - 1:
            w = rng.normal(0.0, np.sqrt(2.0 / (9 * ci)), size=(co, ci, 3, 3))
        else:
            w = np.zeros((co, ci, 3, 3))
        parts += [w.ravel(), np.zeros(co)]
    parts += [np.zeros(3 * K * C_HID), np.zeros(3 * K)]
    return np.concatenate(parts).astype(np.float32)


class PairStore:
    """Training pairs resident in device memory: (frame_t, u_{t-1}, du_t, db_t)."""

    def __init__(self):
        self.frames, self.u_prev, self.du, self.db = [], [], [], []

    def __len__(self):
        return len(self.frames)

    def add_clip(self, clip, G: int, P: int, temporal: bool = True):
        """Decompose the clip with the plain schedule and keep a pair per frame t >= 1."""
        import torch
        W, H, K = clip.width, clip.height, clip.K
        s = Solver(W, H, default_params(K, gn_iters=G, pcg_iters=P, temporal=int(temporal)))
        s.set_base_colors(clip.b_init)
        prev_u, prev_b = None, None
        frames = torch.from_numpy(np.ascontiguousarray(clip.frames)).cuda()
        ids = torch.from_numpy(np.ascontiguousarray(clip.ids)).cuda()
        for t in range(clip.nframes):
            b, _ = s.decompose_frame(frames[t], ids[t])
            u, _ = s.get_state()
            if prev_u is not None:
                self.frames.append(frames[t].clone())
                self.u_prev.append(prev_u)
                self.du.append(u - prev_u)
                self.db.append((np.asarray(b) - prev_b).astype(np.float32).reshape(-1))
            prev_u, prev_b = u, np.asarray(b).copy()
        s.close()


def make_training_set(K: int, W: int, H: int, nframes: int, frames_per_clip: int, G: int, P: int,
                      seed0: int, log=None, **clip_kw) -> PairStore:
    """nframes pairs from seeded synthetic clips (seeds seed0, seed0 + 1, ...);
    clip_kw (amp, supersample) match the scenes to the workload's recipe."""
    from scenes import make_clip
    store = PairStore()
    i = 0
    while len(store) < nframes:
        clip = make_clip(W, H, K, frames_per_clip, seed0 + i, **clip_kw)
        store.add_clip(clip, G, P)
        i += 1
        if log:
            log(f"training clip {i}: {len(store)} pairs")
    for name in ("frames", "u_prev", "du", "db"):
        setattr(store, name, getattr(store, name)[:nframes])
    return store


def train(net: Net, store: PairStore, epochs: int, lr: float, w_b: float = 1.0, seed: int = 0, log=None):
    """Adam over the stored pairs in a seeded shuffled order; returns the mean loss per epoch."""
    rng = np.random.Generator(np.random.PCG64(seed))
    hist = []
    for ep in range(epochs):
        order = rng.permutation(len(store))
        tot = 0.0
        t0 = time.perf_counter()
        for j, k in enumerate(order):
            want = j % 50 == 0
            loss = net.train_step(store.frames[k], store.u_prev[k], store.du[k], store.db[k], lr, w_b,
                                  want_loss=want)
            if want:
                tot += loss
        hist.append(tot / max(1, (len(order) + 49) // 50))
        if log:
            log(f"epoch {ep + 1}/{epochs}: mean sampled loss {hist[-1]:.4e} ({time.perf_counter() - t0:.1f} s)")
    return hist


def transfer(net_from: Net, K: int, W: int, H: int) -> Net:
    """A network for frames of W x H with the trained weights of net_from."""
    net = Net(K, W, H)
    net.set_params(net_from.get_params())
    return net


def bench_forward(K: int, W: int, H: int, reps: int = 20) -> float:
    """Milliseconds per network forward pass at W x H (He-initialised weights with a
    live output layer, random inputs on the device)."""
    import torch
    net = Net(K, W, H)
    flat = init_params(K, 1)
    flat[flat == 0] = 0.01
    net.set_params(flat)
    g = torch.Generator(device="cuda").manual_seed(0)
    fr = torch.rand((3, H, W), device="cuda", generator=g)
    u = torch.rand((K + 4, H, W), device="cuda", generator=g)
    uo = torch.empty_like(u)
    for _ in range(3):
        net.forward(fr, u, uo)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        net.lib.gid_net_forward(net.h, net_ptr(fr), net_ptr(u), net_ptr(uo), None)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / reps
    net.close()
    return ms


def bench_train_step(K: int, W: int, H: int, reps: int = 20) -> float:
    """Milliseconds per training step (forward, loss gradient, input and weight
    gradients of every layer, Adam) at W x H on random inputs and targets."""
    import torch
    net = Net(K, W, H)
    flat = init_params(K, 1)
    flat[flat == 0] = 0.01
    net.set_params(flat)
    g = torch.Generator(device="cuda").manual_seed(0)
    fr = torch.rand((3, H, W), device="cuda", generator=g)
    u = torch.rand((K + 4, H, W), device="cuda", generator=g)
    du = 0.01 * torch.randn((K + 4, H, W), device="cuda", generator=g)
    db = np.zeros(3 * K, np.float32)
    for _ in range(3):
        net.train_step(fr, u, du, db, 1e-4, want_loss=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        net.train_step(fr, u, du, db, 1e-4, want_loss=False)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / reps
    net.close()
    return ms


def net_ptr(t):
    from ctypes import c_void_p
    return c_void_p(t.data_ptr())


if __name__ == "__main__":
    import argparse
    ap = argparse.ArgumentParser(description="time the warm-start network's forward pass or training step")
    ap.add_argument("--width", type=int, default=1280)
    ap.add_argument("--height", type=int, default=720)
    ap.add_argument("--K", type=int, default=8)
    ap.add_argument("--reps", type=int, default=20)
    ap.add_argument("--train", action="store_true", help="time a training step instead of a forward pass")
    a = ap.parse_args()
    if a.train:
        print(f"network training step {a.width}x{a.height} K={a.K}: "
              f"{bench_train_step(a.K, a.width, a.height, a.reps):.3f} ms", flush=True)
    else:
        print(f"network forward {a.width}x{a.height} K={a.K}: {bench_forward(a.K, a.width, a.height, a.reps):.3f} ms",
              flush=True)
