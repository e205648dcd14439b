"""Pins of the oracle's re-synthesis (Sec. 8.4) against the scene renderer,
an independent statement of the image-formation model of Sec. 4: rebuilding a
noise-free frame from its true layers gives the frame; recolouring one base
colour (its indirect light and the reflectance of its regions) gives the scene
rendered with that colour replaced; dropping a colour's indirect layer gives
the scene rendered without that colour's indirect light.  CPU only."""
import numpy as np
import pytest

from oracle.resynthesis import resynthesize
from scenes.generator import _render, _scene

W, H, K, SEED = 80, 50, 4, 31


def _layers(sc, t=0):
    img, ids, R, T = _render(sc, W, H, K, t, False, False)
    return img, ids, np.concatenate([R, T])


def test_rebuild_from_true_layers_is_the_frame():
    sc = _scene(W, H, K, SEED, 0.3, False)
    img, ids, L = _layers(sc, 2)
    out = resynthesize(L, sc["b"])
    assert np.abs(out - img).max() <= 1e-14


def test_recolouring_equals_rendering_with_the_new_colour():
    sc = _scene(W, H, K, SEED, 0.3, False)
    img, ids, L = _layers(sc)
    k = 2
    new = sc["b"].copy()
    new[k] = (0.15, 0.75, 0.4)
    scale = np.ones((K, 3))
    scale[k] = new[k] / sc["b"][k]
    sc2 = dict(sc, b=new)
    ref, _, _, _ = _render(sc2, W, H, K, 0, False, False)
    out = resynthesize(L, new, ids=ids, refl_scale=scale)
    assert np.abs(out - ref).max() <= 1e-14
    assert np.abs(out - img).max() > 1e-2          # the edit shows


@pytest.mark.parametrize("k", [0, 3])
def test_spill_suppression_equals_rendering_without_that_indirect_light(k):
    sc = _scene(W, H, K, SEED, 0.3, False)
    img, ids, L = _layers(sc)
    gain = np.ones(K)
    gain[k] = 0.0
    a = sc["a"].copy()
    a[k] = 0.0
    ref, _, _, _ = _render(dict(sc, a=a), W, H, K, 0, False, False)
    out = resynthesize(L, sc["b"], gain=gain)
    assert np.abs(out - ref).max() <= 1e-14
