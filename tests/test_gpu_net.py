"""The learned warm-start network on the GPU versus its FP64 reference, through the C ABI.

Single layers are fed BF16 values, so every product is exact in FP32 and the
only difference to the FP64 reference is the FP32 summation: 2e-6 of the
output's largest magnitude (measured ~2e-7).  The whole network rounds every stored activation
(and, in the backward pass, every stored gradient) to BF16 on both sides; a
value whose FP32 and FP64 sums fall on different sides of a BF16 rounding
boundary moves by one BF16 step (2^-8 relative), so whole-network outputs and
gradients are compared by relative Frobenius norm (measured on the 80 x 24
case: du 9e-4, db 7e-6, gradients at most 3e-4; the bars below are about 3x).
"""
import sys

import numpy as np
import pytest

import oracle.warmstart as WS

pytestmark = pytest.mark.gpu


def _say(*m):
    print("[gpu-case]", *m, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    if not _t.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1908_01961_amd as G
    G.load_library()
    return _t


def _layers(K):
    n = K + 4
    cin = [3 + n] + [32] * 5
    cout = [32] * 5 + [n]
    return n, cin, cout


def dict_to_flat(p, K):
    """The parameter vector in the library's documented order."""
    parts = []
    for l in range(WS.N_CONV):
        parts += [p[f"w{l}"].ravel(), p[f"b{l}"].ravel()]
    parts += [p["hw"].ravel(), p["hb"].ravel()]
    return np.concatenate(parts).astype(np.float32)


def flat_to_dict(flat, K):
    n, cin, cout = _layers(K)
    p, o = {}, 0
    for l in range(WS.N_CONV):
        m = cout[l] * cin[l] * 9
        p[f"w{l}"] = flat[o:o + m].reshape(cout[l], cin[l], 3, 3).astype(np.float64)
        o += m
        p[f"b{l}"] = flat[o:o + cout[l]].astype(np.float64)
        o += cout[l]
    p["hw"] = flat[o:o + 3 * K * 32].reshape(3 * K, 32).astype(np.float64)
    o += 3 * K * 32
    p["hb"] = flat[o:o + 3 * K].astype(np.float64)
    return p


def _random_params(K, seed, scale_last=1.0):
    """He-scaled random parameters with a live output layer and head (FP32 values)."""
    rng = np.random.default_rng(seed)
    n, cin, cout = _layers(K)
    p = {}
    for l in range(WS.N_CONV):
        std = np.sqrt(2.0 / (9 * cin[l])) * (scale_last if l == WS.N_CONV - 1 else 1.0)
        p[f"w{l}"] = rng.normal(0.0, std, size=(cout[l], cin[l], 3, 3))
        p[f"b{l}"] = rng.normal(0.0, 0.05, size=cout[l])
    p["hw"] = rng.normal(0.0, 0.2, size=(3 * K, 32))
    p["hb"] = rng.normal(0.0, 0.02, size=3 * K)
    flat = dict_to_flat(p, K)
    return flat, flat_to_dict(flat, K)


def _inputs(K, W, H, seed):
    rng = np.random.default_rng(seed)
    n = K + 4
    frame = rng.uniform(0.05, 0.95, size=(3, H, W)).astype(np.float32)
    u = np.empty((n, H, W), np.float32)
    u[:3] = rng.uniform(-1.5, -0.1, size=(3, H, W))
    u[3] = rng.uniform(0.3, 1.0, size=(H, W))
    u[4:] = rng.uniform(-0.02, 0.1, size=(K, H, W))
    return frame, u


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(1e-30, np.linalg.norm(b)))


# ---------------------------------------------------------------- single layers

@pytest.mark.parametrize("layer", [0, 2, 5])
def test_layer_forward_matches_reference(torch, layer):
    import paper_1908_01961_amd as G
    K, W, H = 4, 70, 9                      # a ragged 64-pixel strip and a ragged 4-row group
    n, cin, cout = _layers(K)
    flat, p = _random_params(K, 10 + layer)
    net = G.Net(K, W, H)
    net.set_params(flat)
    rng = np.random.default_rng(20 + layer)
    x = np.zeros((H, W, 32), np.float32)
    x[:, :, :cin[layer]] = rng.normal(0, 1, size=(H, W, cin[layer]))
    xb = torch.from_numpy(x).to(torch.bfloat16).cuda()
    out = torch.empty((H, W, 32), dtype=torch.float32, device="cuda")
    net.layer_forward(layer, xb, out)
    xr = xb.float().cpu().numpy().astype(np.float64).transpose(2, 0, 1)[:cin[layer]]
    ref = WS.conv3x3(xr, WS.bf16_round(p[f"w{layer}"]), p[f"b{layer}"])          # (cout, H, W)
    got = out.cpu().numpy().transpose(2, 0, 1)[:cout[layer]]
    err = np.abs(got - ref).max() / np.abs(ref).max()
    _say(f"layer {layer} forward: max err / max |ref| = {err:.2e}")
    assert err <= 2e-6
    net.close()


@pytest.mark.parametrize("layer", [0, 3, 5])
def test_layer_weight_gradient_matches_reference(torch, layer):
    import paper_1908_01961_amd as G
    K, W, H = 4, 70, 9
    n, cin, cout = _layers(K)
    flat, _ = _random_params(K, 30)
    net = G.Net(K, W, H)
    net.set_params(flat)
    rng = np.random.default_rng(40 + layer)
    x = np.zeros((H, W, 32), np.float32)
    x[:, :, :cin[layer]] = rng.normal(0, 1, size=(H, W, cin[layer]))
    gy = np.zeros((H, W, 32), np.float32)
    gy[:, :, :cout[layer]] = rng.normal(0, 1, size=(H, W, cout[layer]))
    xb = torch.from_numpy(x).to(torch.bfloat16).cuda()
    gb_ = torch.from_numpy(gy).to(torch.bfloat16).cuda()
    gw, gb = net.layer_wgrad(layer, xb, gb_, cin[layer], cout[layer])
    xr = xb.float().cpu().numpy().astype(np.float64).transpose(2, 0, 1)[:cin[layer]]
    gr = gb_.float().cpu().numpy().astype(np.float64).transpose(2, 0, 1)[:cout[layer]]
    _, gw_ref, gb_ref = WS.conv3x3_backward(xr, np.zeros((cout[layer], cin[layer], 3, 3)), gr)
    ew = np.abs(gw - gw_ref).max() / np.abs(gw_ref).max()
    eb = np.abs(gb - gb_ref).max() / np.abs(gb_ref).max()
    _say(f"layer {layer} wgrad: weights {ew:.2e}, bias {eb:.2e}")
    assert ew <= 2e-6 and eb <= 2e-6
    net.close()


# ---------------------------------------------------------------- whole network

CASE = dict(K=4, W=80, H=24)
NLAYERS = 6      # conv layers, each storing BF16 activations (and, backward, BF16 gradients)


def test_forward_matches_reference(torch):
    import paper_1908_01961_amd as G
    K, W, H = CASE["K"], CASE["W"], CASE["H"]
    flat, p = _random_params(K, 50)
    frame, u = _inputs(K, W, H, 51)
    net = G.Net(K, W, H)
    net.set_params(flat)
    uo = torch.empty((K + 4, H, W), dtype=torch.float32, device="cuda")
    db = net.forward(_dev(torch, frame), _dev(torch, u), uo)
    du = uo.cpu().numpy().astype(np.float64) - u
    x = np.concatenate([frame, u]).astype(np.float64)
    du_ref, db_ref, _ = WS.forward(p, x)
    e_u, e_b = _rel(du, du_ref), _rel(db, db_ref)
    # element by element: one BF16 step (2^-8 relative) of the element plus one
    # step of the output's RMS per layer.  Each of the six layers stores its
    # activations in BF16; an activation whose FP32 (GPU) and FP64 (oracle) sums
    # straddle a rounding boundary moves by one step, and the later layers carry
    # that change to the output at about the activations' scale.
    step = 2.0 ** -8
    bu = step * (np.abs(du_ref) + NLAYERS * np.sqrt((du_ref ** 2).mean()))
    bb = step * (np.abs(db_ref) + NLAYERS * np.sqrt((db_ref ** 2).mean()))
    ru = float((np.abs(du - du_ref) / bu).max())
    rb = float((np.abs(db - db_ref) / bb).max())
    _say(f"forward: |du - ref| / |ref| = {e_u:.2e}, |db - ref| / |ref| = {e_b:.2e}, "
         f"max |du - ref| = {np.abs(du - du_ref).max():.2e} (max |ref| {np.abs(du_ref).max():.2e}); "
         f"element error / one-BF16-step bound: du {ru:.3f}, db {rb:.3f}")
    assert e_u <= 3e-3 and e_b <= 3e-5
    assert ru <= 1.0 and rb <= 1.0
    net.close()


def test_gradients_match_reference(torch):
    import paper_1908_01961_amd as G
    K, W, H = CASE["K"], CASE["W"], CASE["H"]
    flat, p = _random_params(K, 60)
    frame, u = _inputs(K, W, H, 61)
    rng = np.random.default_rng(62)
    du_t = (0.05 * rng.normal(size=u.shape)).astype(np.float32)
    db_t = (0.05 * rng.normal(size=3 * K)).astype(np.float32)
    wb = 2.0
    net = G.Net(K, W, H)
    net.set_params(flat)
    g, loss = net.gradients(_dev(torch, frame), _dev(torch, u), _dev(torch, du_t), db_t, wb)
    gd = flat_to_dict(g, K)
    x = np.concatenate([frame, u]).astype(np.float64)
    du, dbv, cache = WS.forward(p, x)
    loss_ref, g_du, g_db = WS.mse_loss(du, dbv, du_t.astype(np.float64), db_t.astype(np.float64), wb)
    gref = WS.backward(p, cache, g_du, g_db)
    _say(f"loss gpu {loss:.8e} ref {loss_ref:.8e}")
    assert loss == pytest.approx(loss_ref, rel=1e-5)
    step = 2.0 ** -8
    for k in gref:
        e = _rel(gd[k], gref[k])
        # element by element, as for the forward pass: the backward pass stores the
        # loss gradient and every layer's input gradient in BF16 too
        bound = step * (np.abs(gref[k]) + NLAYERS * np.sqrt((gref[k] ** 2).mean()))
        r = float((np.abs(gd[k] - gref[k]) / bound).max())
        _say(f"  grad {k}: rel {e:.2e} (|ref| {np.linalg.norm(gref[k]):.2e}), element error / bound {r:.3f}")
        assert e <= 1e-3, k
        assert r <= 1.0, k
    net.close()


def test_adam_step_matches_reference(torch):
    import paper_1908_01961_amd as G
    K, W, H = CASE["K"], CASE["W"], CASE["H"]
    flat, p = _random_params(K, 70)
    frame, u = _inputs(K, W, H, 71)
    rng = np.random.default_rng(72)
    du_t = (0.05 * rng.normal(size=u.shape)).astype(np.float32)
    db_t = (0.05 * rng.normal(size=3 * K)).astype(np.float32)
    lr = 1e-3
    net = G.Net(K, W, H)
    net.set_params(flat)
    g, _ = net.gradients(_dev(torch, frame), _dev(torch, u), _dev(torch, du_t), db_t, 1.0)
    net.train_step(_dev(torch, frame), _dev(torch, u), _dev(torch, du_t), db_t, lr)
    after = net.get_params()
    # the oracle's Adam step from the oracle's own gradient of the same loss
    x = np.concatenate([frame, u]).astype(np.float64)
    du, dbv, cache = WS.forward(p, x)
    _, g_du, g_db = WS.mse_loss(du, dbv, du_t.astype(np.float64), db_t.astype(np.float64), 1.0)
    gref = WS.backward(p, cache, g_du, g_db)
    pd = {k: vv.copy() for k, vv in flat_to_dict(flat, K).items()}
    m = {k: np.zeros_like(vv) for k, vv in pd.items()}
    v = {k: np.zeros_like(vv) for k, vv in pd.items()}
    WS.adam_step(pd, gref, m, v, 1, lr)
    ref = dict_to_flat(pd, K).astype(np.float64)
    # Adam's first step is lr g / (|g| + eps) per parameter: it agrees wherever the
    # two gradients agree in sign and are well above eps; elsewhere (gradients
    # within their own difference of zero) the step is bounded by 2 lr
    gflat = dict_to_flat(gref, K).astype(np.float64)
    gdiff = np.abs(g.astype(np.float64) - gflat)
    sure = np.abs(gflat) > 10.0 * gdiff + 1e-6
    err = np.abs(after - ref)
    _say(f"adam from the oracle's gradient: max |p_gpu - p_ref| = {err[sure].max():.2e} on {int(sure.sum())} of "
         f"{sure.size} parameters with a certain gradient sign, {err[~sure].max() if (~sure).any() else 0.0:.2e} "
         f"on the rest (step size {lr})")
    assert sure.mean() > 0.9
    assert err[sure].max() <= 1e-6
    assert err.max() <= 2.0 * lr + 1e-6
    net.close()


def test_training_reduces_the_loss(torch):
    import paper_1908_01961_amd as G
    K, W, H = CASE["K"], CASE["W"], CASE["H"]
    flat, _ = _random_params(K, 80, scale_last=0.1)
    frame, u = _inputs(K, W, H, 81)
    # a target the network can represent: a smooth function of the input
    du_t = (0.1 * np.tanh(u - u.mean(axis=(1, 2), keepdims=True))).astype(np.float32)
    db_t = np.full(3 * K, 0.02, np.float32)
    net = G.Net(K, W, H)
    net.set_params(flat)
    f, uu, t = _dev(torch, frame), _dev(torch, u), _dev(torch, du_t)
    losses = [net.train_step(f, uu, t, db_t, 2e-3) for _ in range(60)]
    _say(f"training: loss {losses[0]:.3e} -> {losses[-1]:.3e}")
    assert losses[-1] < 0.3 * losses[0]
    net.close()


# -------------------------------------------------- many tiles per workgroup

# 6 x 260 = 1560 tiles of 4 rows x 64 pixels (the last strip 54 pixels wide, the
# last row group 3 rows high): more than the resident grid of two workgroups per
# compute unit, so that each workgroup walks several tiles.
BIG = dict(K=4, W=374, H=1039)


def test_conv_launch_shapes_are_bit_identical(torch):
    """The convolution's launch shape -- the resident grid (several tiles per
    workgroup, the next tile's input staged while the current one computes), one
    workgroup per tile, a single workgroup walking every tile, an odd count --
    leaves the forward outputs, the gradients and the loss unchanged bit for bit:
    a tile's arithmetic and its partial-sum slots do not depend on which
    workgroup computes it."""
    import paper_1908_01961_amd as G
    K, W, H = BIG["K"], BIG["W"], BIG["H"]
    ntiles = -(-W // 64) * -(-H // 4)
    flat, _ = _random_params(K, 90)
    frame, u = _inputs(K, W, H, 91)
    rng = np.random.default_rng(92)
    du_t = (0.05 * rng.normal(size=u.shape)).astype(np.float32)
    db_t = (0.05 * rng.normal(size=3 * K)).astype(np.float32)
    net = G.Net(K, W, H)
    net.set_params(flat)
    f, uu, t = _dev(torch, frame), _dev(torch, u), _dev(torch, du_t)
    runs = {}
    for wg in (0, ntiles, 1, 7):
        net.set_conv_workgroups(wg)
        uo = torch.empty((K + 4, H, W), dtype=torch.float32, device="cuda")
        db = np.array(net.forward(f, uu, uo), np.float32)
        g, loss = net.gradients(f, uu, t, db_t, 2.0)
        runs[wg] = (uo.cpu().numpy(), db, np.array(g, np.float32), float(loss))
        _say(f"conv workgroups {wg or 'resident'} of {ntiles} tiles: loss {loss:.10e}")
    u0, db0, g0, l0 = runs[0]
    assert np.isfinite(u0).all() and np.isfinite(g0).all()
    for wg, (uw, dbw, gw, lw) in runs.items():
        assert np.array_equal(uw, u0), wg
        assert np.array_equal(dbw, db0), wg
        assert np.array_equal(gw, g0), wg
        assert lw == l0, wg
    with pytest.raises(G.GidError):
        net.set_conv_workgroups(-1)
    net.close()


def test_forward_at_full_size_matches_reference_on_sampled_pixels(torch):
    """1920 x 1080, K = 10 (the warm start's size in the benchmark; the resident
    grid walks 8100 tiles): du at sampled pixels against the oracle network
    applied to the pixel's 13 x 13 neighbourhood, the receptive field of six 3 x 3
    layers (clipped at the frame, where both sides pad with zeros).  Samples: the
    frame's corners and edges, pixels on both sides of strip and row-group
    boundaries, and random pixels."""
    import paper_1908_01961_amd as G
    K, W, H = 10, 1920, 1080
    flat, p = _random_params(K, 95)
    frame, u = _inputs(K, W, H, 96)
    net = G.Net(K, W, H)
    net.set_params(flat)
    uo = torch.empty((K + 4, H, W), dtype=torch.float32, device="cuda")
    net.forward(_dev(torch, frame), _dev(torch, u), uo)
    got_all = uo.cpu().numpy()
    net.close()
    xs = [0, 1, 63, 64, 65, 127, 128, 959, 960, 1855, 1856, 1918, 1919]
    ys = [0, 1, 3, 4, 5, 7, 8, 539, 540, 1075, 1076, 1078, 1079]
    rng = np.random.default_rng(97)
    pts = [(y, x) for y in ys for x in xs] + list(zip(rng.integers(0, H, 120).tolist(), rng.integers(0, W, 120).tolist()))
    x_full = np.concatenate([frame, u]).astype(np.float64)
    ref = np.empty((len(pts), K + 4))
    got = np.empty((len(pts), K + 4))
    for j, (y, x) in enumerate(pts):
        y0, y1, x0, x1 = max(0, y - 6), min(H, y + 7), max(0, x - 6), min(W, x + 7)
        d, _, _ = WS.forward(p, x_full[:, y0:y1, x0:x1])
        ref[j] = d[:, y - y0, x - x0]
        got[j] = got_all[:, y, x].astype(np.float64) - u[:, y, x]
    # the whole-network bound of the 80 x 24 case, the RMS taken over the samples
    step = 2.0 ** -8
    bound = step * (np.abs(ref) + NLAYERS * np.sqrt((ref ** 2).mean()))
    r = float((np.abs(got - ref) / bound).max())
    _say(f"1920x1080 K=10 forward, {len(pts)} sampled pixels: max |du - ref| = {np.abs(got - ref).max():.2e} "
         f"(max |ref| {np.abs(ref).max():.2e}); element error / one-BF16-step bound {r:.3f}")
    assert r <= 1.0
