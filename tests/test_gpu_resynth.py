"""Re-synthesis (Sec. 8.4) on the GPU against the oracle, through the C ABI,
on the true layers of seeded scenes: a plain rebuild, a recolouring with a
reflectance edit, spill suppression, ragged sizes that take the one-pixel path
and ids outside [0, K).  FP32 arithmetic against FP64: every element within
2e-6 of the sum of the magnitudes it is formed from."""
import numpy as np
import pytest

from oracle.resynthesis import resynthesize as oracle_resynth
from scenes import make_clip

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    if not _t.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1908_01961_amd as G
    G.load_library()
    return _t


def _layers(c, t=0):
    return np.concatenate([np.exp(c.gt_r[t].astype(np.float64)), c.gt_T[t]]).astype(np.float32)


def _bound(L, b, gain, ids, scale):
    """Sum of the magnitudes of the terms of every output element."""
    K = L.shape[0] - 4
    Lf = np.abs(L.astype(np.float64))
    g = np.ones(K) if gain is None else np.abs(np.asarray(gain, np.float64))
    S = np.repeat(Lf[3][None], 3, axis=0)
    for k in range(K):
        S = S + (g[k] * np.abs(b[k]))[:, None, None] * Lf[4 + k][None]
    R = Lf[:3]
    if ids is not None:
        s = np.abs(np.asarray(scale, np.float64))
        ok = ids < K
        R = R * np.where(ok[None], s[np.minimum(ids, K - 1)].transpose(2, 0, 1), 1.0)
    return R * S


def _reference(L, b, gain, ids, scale):
    K = L.shape[0] - 4
    if ids is None or np.all(ids < K):
        return oracle_resynth(L, b, gain, ids, scale)
    # ids outside [0, K) keep their reflectance: apply the edit with a unit row
    # for them, then recombine without a further edit
    wide = np.vstack([np.asarray(scale, np.float64), np.ones((1, 3))])
    R = L[:3].astype(np.float64) * wide[np.where(ids < K, ids, K)].transpose(2, 0, 1)
    return oracle_resynth(np.concatenate([R, L[3:].astype(np.float64)]), b, gain)


def _check(torch, L, b, gain=None, ids=None, scale=None, label=""):
    import paper_1908_01961_amd as G
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    out = G.resynthesize(dev(L), b, gain, None if ids is None else dev(ids), scale).cpu().numpy()
    ref = _reference(L, b, gain, ids, scale)
    err = np.abs(out - ref)
    bound = 2e-6 * _bound(L, np.asarray(b), gain, ids, scale) + 1e-30
    print(f"[gpu-case] resynth {label}: max |err| {err.max():.2e}, max err / bound {(err / bound).max():.3f}",
          flush=True)
    assert np.all(err <= bound)


def test_plain_rebuild_and_edits(torch):
    c = make_clip(320, 240, 6, 1, 71, amp=0.35)
    L = _layers(c)
    _check(torch, L, c.b_gt, label="rebuild 320x240 K=6")
    new = c.b_gt.copy()
    new[2] = (0.1, 0.8, 0.3)
    scale = np.ones((6, 3), np.float32)
    scale[2] = (new[2] / c.b_gt[2]).astype(np.float32)
    _check(torch, L, new, ids=c.ids[0], scale=scale, label="recolour colour 2")
    gain = np.ones(6, np.float32)
    gain[4] = 0.0
    _check(torch, L, c.b_gt, gain=gain, label="spill of colour 4 removed")


@pytest.mark.parametrize("W,H,K", [(1, 1, 1), (33, 17, 16), (127, 5, 3), (1920, 1080, 10)])
def test_sizes_and_ids_out_of_range(torch, W, H, K):
    c = make_clip(W, H, K, 1, 90 + K)
    L = _layers(c)
    ids = c.ids[0].copy()
    ids.flat[:: 7] = 200                      # outside [0, K): reflectance kept
    rng = np.random.default_rng(K)
    scale = rng.uniform(0.5, 1.5, size=(K, 3)).astype(np.float32)
    gain = rng.uniform(0.0, 2.0, size=K).astype(np.float32)
    _check(torch, L, c.b_gt, gain=gain, ids=ids, scale=scale, label=f"{W}x{H} K={K}")
