"""FP64 reference of the learned warm-start network (test infrastructure only).

The network is not in the paper (which names learned priors only as future
work, Sec. 9); its definition is this project's: six 3x3 convolutions with 32
channels, ReLU after the first five, zero padding, stride 1.

  input   x = (I_t, u_{t-1}): 3 + n channels, n = K + 4
  L1      conv c_in -> 32, ReLU
  L2..L5  conv 32 -> 32, ReLU
  L6      conv 32 -> n          output: u_t = u_{t-1} + L6
  head    global average of the L5 features (32) -> linear 32 -> 3K: b_t = b_{t-1} + head

Weights and activations are stored in BF16 (round to nearest even) and every
product is accumulated in higher precision; this reference rounds exactly where
the GPU kernels do (weights, network input, every stored activation) and
accumulates in FP64.  Layouts: activations (C, H, W); conv weights
(C_out, C_in, 3, 3); tap (dy, dx) reads x[c, y + dy - 1, x + dx - 1].
"""
from __future__ import annotations

import numpy as np

C_HID = 32
N_CONV = 6


def bf16_round(x: np.ndarray) -> np.ndarray:
    """Round float values to the nearest BF16 (ties to even), returned as float64."""
    a = np.ascontiguousarray(np.asarray(x, np.float32))
    u = a.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    nan = np.isnan(a)
    out = (r & 0xFFFFFFFF).astype(np.uint32).view(np.float32).astype(np.float64)
    out[nan] = np.nan
    return out


def conv3x3(x: np.ndarray, w: np.ndarray, b: np.ndarray) -> np.ndarray:
    """y[o] = b[o] + sum_{c, dy, dx} w[o, c, dy, dx] x[c, . + dy - 1, . + dx - 1], zero padded."""
    C, H, W = x.shape
    xp = np.zeros((C, H + 2, W + 2))
    xp[:, 1:-1, 1:-1] = x
    y = np.zeros((w.shape[0], H, W)) + np.asarray(b, np.float64)[:, None, None]
    for dy in range(3):
        for dx in range(3):
            y += np.einsum("oc,chw->ohw", w[:, :, dy, dx], xp[:, dy:dy + H, dx:dx + W])
    return y


def conv3x3_backward(x: np.ndarray, w: np.ndarray, gy: np.ndarray):
    """Gradients of sum(gy * conv3x3(x, w, b)) with respect to x, w and b."""
    C, H, W = x.shape
    xp = np.zeros((C, H + 2, W + 2))
    xp[:, 1:-1, 1:-1] = x
    gw = np.zeros_like(w, dtype=np.float64)
    gxp = np.zeros_like(xp)
    for dy in range(3):
        for dx in range(3):
            gw[:, :, dy, dx] = np.einsum("ohw,chw->oc", gy, xp[:, dy:dy + H, dx:dx + W])
            gxp[:, dy:dy + H, dx:dx + W] += np.einsum("oc,ohw->chw", w[:, :, dy, dx], gy)
    return gxp[:, 1:-1, 1:-1], gw, gy.sum(axis=(1, 2))


def init_params(n: int, K: int, seed: int) -> dict:
    """He-style initialisation (BF16-rounded conv weights, zero biases); the last
    conv and the colour head start at zero so the untrained net is the identity."""
    rng = np.random.Generator(np.random.PCG64(seed))
    cin = 3 + n
    chans = [cin] + [C_HID] * 5 + [n]
    p = {}
    for l in range(N_CONV):
        ci, co = chans[l], chans[l + 1]
        std = np.sqrt(2.0 / (9 * ci))
        w = rng.normal(0.0, std, size=(co, ci, 3, 3)) if l < N_CONV - 1 else np.zeros((co, ci, 3, 3))
        p[f"w{l}"] = w
        p[f"b{l}"] = np.zeros(co)
    p["hw"] = np.zeros((3 * K, C_HID))
    p["hb"] = np.zeros(3 * K)
    return p


def forward(p: dict, x: np.ndarray, rnd=bf16_round):
    """Return (delta_u, delta_b, cache).  x is rounded to BF16 on entry; the
    outputs of L1..L5 are rounded to BF16 after the ReLU (they are stored
    activations); L6 and the head stay in higher precision.  rnd replaces the
    rounding (identity for derivative checks)."""
    acts = [rnd(x)]
    pre = []
    h = acts[0]
    for l in range(N_CONV):
        z = conv3x3(h, rnd(p[f"w{l}"]), p[f"b{l}"])
        pre.append(z)
        if l < N_CONV - 1:
            h = rnd(np.maximum(z, 0.0))
            acts.append(h)
    du = pre[-1]
    pooled = acts[5].mean(axis=(1, 2))
    db = p["hw"] @ pooled + p["hb"]
    return du, db, dict(acts=acts, pre=pre, pooled=pooled)


def backward(p: dict, cache: dict, g_du: np.ndarray, g_db: np.ndarray, rnd=bf16_round) -> dict:
    """Gradients of a scalar loss with d(loss)/d(delta_u) = g_du and
    d(loss)/d(delta_b) = g_db.  Rounding steps of the forward pass are treated
    as identity (straight-through); the gradient tensors that are stored and fed
    to the next contraction -- g_du and each layer's input gradient after the
    ReLU mask -- are rounded by rnd where the GPU stores them in BF16."""
    acts, pre = cache["acts"], cache["pre"]
    g = {}
    g["hw"] = np.outer(g_db, cache["pooled"])
    g["hb"] = g_db.copy()
    H, W = acts[0].shape[1:]
    g_pool = p["hw"].T @ g_db                              # (32,)
    gy = rnd(g_du)
    for l in range(N_CONV - 1, -1, -1):
        gx, gw, gb = conv3x3_backward(acts[l], rnd(p[f"w{l}"]), gy)
        g[f"w{l}"], g[f"b{l}"] = gw, gb
        if l == 0:
            break
        gx = gx.copy()
        if l == 5:
            gx += g_pool[:, None, None] / (H * W)          # the head reads the L5 features
        gy = rnd(gx * (pre[l - 1] > 0.0))                   # through the ReLU of layer l-1
    return g


def mse_loss(du, db, t_du, t_db, w_b: float = 1.0):
    """0.5 * mean((du - t_du)^2) + 0.5 * w_b * mean((db - t_db)^2) and its gradients."""
    n1, n2 = du.size, db.size
    e1, e2 = du - t_du, db - t_db
    loss = 0.5 * (e1 ** 2).sum() / n1 + 0.5 * w_b * (e2 ** 2).sum() / n2
    return loss, e1 / n1, w_b * e2 / n2


def adam_step(p: dict, g: dict, m: dict, v: dict, t: int, lr: float, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update in place (FP32 master weights on the GPU; FP64 here)."""
    for k in p:
        m[k] = b1 * m[k] + (1 - b1) * g[k]
        v[k] = b2 * v[k] + (1 - b2) * g[k] ** 2
        mh = m[k] / (1 - b1 ** t)
        vh = v[k] / (1 - b2 ** t)
        p[k] = p[k] - lr * mh / (np.sqrt(vh) + eps)
