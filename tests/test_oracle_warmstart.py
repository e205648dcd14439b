"""Pins of the FP64 reference of the learned warm-start network: convolution
against scipy's correlate2d, BF16 rounding against torch's bfloat16, gradients
against central differences, Adam against torch.optim.Adam.  CPU only."""
import numpy as np
import pytest
from scipy.signal import correlate2d

from oracle import warmstart as WS


def test_conv3x3_matches_scipy_correlate2d():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((3, 7, 9))
    w = rng.standard_normal((4, 3, 3, 3))
    b = rng.standard_normal(4)
    y = WS.conv3x3(x, w, b)
    for o in range(4):
        ref = b[o] + sum(correlate2d(x[c], w[o, c], mode="same", boundary="fill") for c in range(3))
        assert np.allclose(y[o], ref, rtol=1e-12, atol=1e-12)


def test_bf16_round_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(1)
    x = np.concatenate([rng.standard_normal(10000) * 10.0 ** rng.integers(-6, 6, 10000),
                        [0.0, -0.0, 1.0, 65504.0, 1e-40]]).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy().astype(np.float64)
    assert np.array_equal(WS.bf16_round(x), ref)


def _loss(p, x, t_du, t_db):
    du, db, cache = WS.forward(p, x, rnd=lambda a: np.asarray(a, np.float64))
    return WS.mse_loss(du, db, t_du, t_db), cache


def test_gradients_match_central_differences():
    n, K, H, W = 5, 1, 5, 6
    rng = np.random.default_rng(2)
    p = WS.init_params(n, K, seed=3)
    for k in p:   # make every parameter non-zero so every path carries gradient
        p[k] = p[k] + 0.05 * rng.standard_normal(p[k].shape)
    x = rng.standard_normal((3 + n, H, W))
    t_du = rng.standard_normal((n, H, W))
    t_db = rng.standard_normal(3 * K)
    ident = lambda a: np.asarray(a, np.float64)
    (loss, g_du, g_db), cache = _loss(p, x, t_du, t_db)
    g = WS.backward(p, cache, g_du, g_db, rnd=ident)
    h = 1e-6
    for key in ("w0", "w3", "w5", "b1", "b5", "hw", "hb"):
        flat = p[key].reshape(-1)
        for j in rng.choice(flat.size, size=min(6, flat.size), replace=False):
            old = flat[j]
            flat[j] = old + h
            (lp, _, _), _ = _loss(p, x, t_du, t_db)
            flat[j] = old - h
            (lm, _, _), _ = _loss(p, x, t_du, t_db)
            flat[j] = old
            fd = (lp - lm) / (2 * h)
            an = g[key].reshape(-1)[j]
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(fd)), (key, j, fd, an)


def test_untrained_net_is_identity():
    n, K = 8, 4
    p = WS.init_params(n, K, seed=1)
    x = np.random.default_rng(4).standard_normal((3 + n, 6, 5))
    du, db, _ = WS.forward(p, x)
    assert np.abs(du).max() == 0 and np.abs(db).max() == 0


def test_adam_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(5)
    p = {"a": rng.standard_normal((3, 4)), "b": rng.standard_normal(5)}
    m = {k: np.zeros_like(v) for k, v in p.items()}
    v = {k: np.zeros_like(v) for k, v in p.items()}
    tp = {k: torch.tensor(x, dtype=torch.float64, requires_grad=True) for k, x in p.items()}
    opt = torch.optim.Adam(list(tp.values()), lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    for t in range(1, 4):
        g = {k: rng.standard_normal(x.shape) for k, x in p.items()}
        WS.adam_step(p, g, m, v, t, lr=1e-2)
        opt.zero_grad()
        for k in tp:
            tp[k].grad = torch.tensor(g[k])
        opt.step()
    for k in p:
        assert np.allclose(p[k], tp[k].detach().numpy(), rtol=1e-12, atol=1e-14)


def test_du_depends_only_on_the_13x13_neighbourhood():
    """Six 3 x 3 layers: du at a pixel is the network applied to the pixel's
    13 x 13 neighbourhood, clipped at the frame (zero padding on both sides), and
    the one-pixel-smaller window does not give it.  The GPU test at full frame
    size checks sampled pixels this way."""
    rng = np.random.default_rng(5)
    K, H, W = 2, 30, 40
    n = K + 4
    chans = [3 + n] + [WS.C_HID] * 5 + [n]
    p = {}
    for l in range(WS.N_CONV):
        p[f"w{l}"] = rng.normal(0.0, np.sqrt(2.0 / (9 * chans[l])), size=(chans[l + 1], chans[l], 3, 3))
        p[f"b{l}"] = rng.normal(0.0, 0.05, size=chans[l + 1])
    p["hw"] = rng.normal(0.0, 0.2, size=(3 * K, WS.C_HID))
    p["hb"] = rng.normal(0.0, 0.02, size=3 * K)
    x = rng.uniform(-1.0, 1.0, size=(3 + n, H, W))
    ident = lambda a: np.asarray(a, np.float64)   # noqa: E731
    du, _, _ = WS.forward(p, x, rnd=ident)
    for y, xx in [(0, 0), (0, 39), (29, 0), (29, 39), (3, 20), (15, 6), (15, 33), (14, 20), (22, 7)]:
        y0, y1, x0, x1 = max(0, y - 6), min(H, y + 7), max(0, xx - 6), min(W, xx + 7)
        d, _, _ = WS.forward(p, x[:, y0:y1, x0:x1], rnd=ident)
        assert np.allclose(d[:, y - y0, xx - x0], du[:, y, xx], rtol=1e-12, atol=1e-12)
    y, xx = 15, 20
    d, _, _ = WS.forward(p, x[:, y - 5:y + 6, xx - 5:xx + 6], rnd=ident)
    assert not np.allclose(d[:, 5, 5], du[:, y, xx], rtol=1e-6, atol=1e-9)
