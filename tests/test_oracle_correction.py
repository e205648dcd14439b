"""Pins of the oracle's misclustering correction (Sec. 5.2.2): the region
sparsity by hand, and the paper's claim that the true reflectance gives the
sparsest indirect layers, on scenes with a region mislabelled.  CPU only."""
import numpy as np
import pytest

import oracle as O
from oracle.correction import correct_region, region_sparsity
from scenes import make_clip

P = O.default_params()


def test_region_sparsity_hand_value():
    u = np.zeros((7, 2, 3))          # K = 3
    u[4] = [[0.1, -0.2, 0.0], [0.0, 0.0, 0.5]]
    u[5, 0, 0] = 0.3
    u[6, 1, 2] = -0.05
    u[3] = 9.0                       # T_0 does not count
    region = np.array([[1, 1, 0], [0, 0, 1]], bool)
    # lambda_is (|0.1| + |-0.2| + |0.3| + |0.5| + |-0.05|) = 3 * 1.15
    assert region_sparsity(u, region, P) == pytest.approx(3 * 1.15, rel=1e-14)


def _mislabelled(seed, true=0, wrong=1):
    c = make_clip(48, 32, 3, 1, seed, amp=0.0, supersample=False)
    ids = c.ids[0].astype(np.int64)
    region = ids == true
    return c, np.where(region, wrong, ids), region


@pytest.mark.parametrize("seed", [300, 302, 303, 304])
def test_true_reflectance_gives_the_sparsest_layers(seed):
    """A region of colour 0 labelled with colour 1: trying every colour, the
    true one explains the region with the sparsest indirect light (the
    region is lit by direct light only) and is chosen."""
    c, wrong, region = _mislabelled(seed)
    best, sp, fixed = correct_region(c.frames[0], wrong, region, c.b_gt, P, 3, 8)
    assert best == 0
    assert sp[0] < min(sp[1:])
    assert np.array_equal(fixed, c.ids[0])


def test_a_correct_label_is_kept():
    c = make_clip(48, 32, 3, 1, 302, amp=0.0, supersample=False)
    ids = c.ids[0].astype(np.int64)
    region = ids == 2
    best, sp, fixed = correct_region(c.frames[0], ids, region, c.b_gt, P, 3, 8)
    assert best == 2 and np.array_equal(fixed, ids)
