"""Misclustering correction (Sec. 5.2.2) on the GPU against the oracle, through
the C ABI.  Each candidate's region sparsity is a sum of |T_k| over the region,
so the layer bar (1e-3 per element) bounds its difference by
lambda_is * |region| * K * 1e-3; the chosen colour must be the oracle's
wherever the oracle's margin between its best and second-best candidates
exceeds twice that bound, and the corrected ids then match bit for bit."""
import sys

import numpy as np
import pytest

import oracle as O
from oracle.correction import correct_region as oracle_correct
from scenes import make_clip

pytestmark = pytest.mark.gpu
P32 = O.default_params(state_precision="f32")


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    if not _t.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1908_01961_amd as G
    G.load_library()
    return _t


def _case(torch, c, ids, region, G_=3, P_=8, label=""):
    import paper_1908_01961_amd as G
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    prm = G.default_params(c.K, gn_iters=G_, pcg_iters=P_)
    best, sp, fixed = G.correct_region(prm, dev(c.frames[0]), dev(ids.astype(np.uint8)), dev(region.astype(np.uint8)),
                                       c.b_gt)
    ob, osp, ofixed = oracle_correct(c.frames[0], ids.astype(np.uint8), region, c.b_gt, P32, G_, P_)
    bound = P32.lam_isparsity * region.sum() * c.K * 1e-3
    srt = np.sort(osp)
    margin = srt[1] - srt[0] if len(srt) > 1 else np.inf
    print(f"[gpu-case] correction {label}: GPU {sp.round(4)} best {best}; oracle {osp.round(4)} best {ob}; "
          f"bound {bound:.3g}, margin {margin:.3g}", flush=True)
    assert np.all(np.abs(sp - osp) <= bound)
    if margin > 2 * bound:
        assert best == ob
        assert np.array_equal(fixed.cpu().numpy(), ofixed)
    return best


@pytest.mark.parametrize("seed", [300, 303])
def test_mislabelled_region_is_corrected_like_the_oracle(torch, seed):
    c = make_clip(48, 32, 3, 1, seed, amp=0.0, supersample=False)
    ids = c.ids[0].astype(np.int64)
    region = ids == 0
    wrong = np.where(region, 1, ids)
    assert _case(torch, c, wrong, region, label=f"48x32 K=3 seed {seed}") == 0


def test_larger_frame_with_indirect_light(torch):
    c = make_clip(160, 120, 5, 1, 311, amp=0.3)
    ids = c.ids[0].astype(np.int64)
    region = ids == 2
    _case(torch, c, np.where(region, 4, ids), region, label="160x120 K=5")


def test_empty_region_keeps_every_id(torch):
    c = make_clip(64, 40, 4, 1, 312)
    ids = c.ids[0].astype(np.int64)
    region = np.zeros_like(ids, bool)
    import paper_1908_01961_amd as G
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    best, sp, fixed = G.correct_region(G.default_params(c.K, gn_iters=2, pcg_iters=4), dev(c.frames[0]),
                                       dev(ids.astype(np.uint8)), dev(region.astype(np.uint8)), c.b_gt)
    assert np.all(sp == 0.0) and best == 0
    assert np.array_equal(fixed.cpu().numpy(), ids)
