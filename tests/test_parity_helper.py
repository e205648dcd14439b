"""The schedule comparison used by the GPU tests, checked on the CPU with
constructed inputs (no GPU, no solver)."""
from types import SimpleNamespace

import numpy as np
import pytest

from parity import LOOSE_BOUND, MAX_OVER_FRAC, TOL_LAYER, compare_frame, nearest_branch_value


def _ref(u, starts=()):
    return SimpleNamespace(u=u, b=np.full((2, 3), 0.4), energy=100.0, starts=list(starts))


def _layers(u):
    return np.concatenate([np.exp(u[:3]), u[3:]])


def test_nearest_branch_value_looks_at_the_pixel_and_its_neighbours_after_step_0():
    st = [np.full((6, 5, 5), 0.5) for _ in range(3)]
    st[0][4, 2, 2] = 1e-12          # the given start state is not a branch point of the schedule
    st[2][5, 2, 3] = -3e-9          # right neighbour, last step
    st[1][3, 0, 0] = 1e-10          # far away
    st[1][1, 2, 2] = 0.0            # r plane: no branch
    assert nearest_branch_value(st, 2, 2) == pytest.approx(3e-9)
    assert nearest_branch_value(st, 4, 4) == 0.5


def test_compare_frame_counts_elements_over_the_bar():
    H, W, n = 100, 100, 6                       # 60000 elements: at most 6 may exceed 1e-3
    u = np.full((n, H, W), 0.25)
    ref = _ref(u)
    say = lambda *a: None
    L = _layers(u)
    rep = compare_frame(L, ref.b, 100.0, ref, say=say)
    assert rep["n_over"] == 0 and rep["max"] == 0.0
    ok = L.copy()
    ok[4, 10, 10:16] += 2e-2                    # 6 elements over the bar, under the loose bound
    rep = compare_frame(ok, ref.b, 100.0, ref, say=say)
    assert rep["n_over"] == 6 and rep["worst"][1:] == (10, 10)
    assert 6 <= MAX_OVER_FRAC * L.size < 7
    bad = ok.copy()
    bad[5, 50, 50] += 2 * TOL_LAYER             # a 7th
    with pytest.raises(AssertionError):
        compare_frame(bad, ref.b, 100.0, ref, say=say)
    worse = L.copy()
    worse[3, 0, 0] += 2 * LOOSE_BOUND           # one element, beyond the loose bound
    with pytest.raises(AssertionError):
        compare_frame(worse, ref.b, 100.0, ref, say=say)
    with pytest.raises(AssertionError):         # reflectance layers are compared as R = exp(r)
        r = L.copy()
        r[0, 1:4, 1:4] *= 1.01
        compare_frame(r, ref.b, 100.0, ref, say=say)
    with pytest.raises(AssertionError):         # energy bar
        compare_frame(L, ref.b, 100.02, ref, say=say)
    with pytest.raises(AssertionError):         # colour bar
        compare_frame(L, ref.b + 2e-3, 100.0, ref, say=say)


def test_compare_frame_energy_may_match_either_storage_variant():
    u = np.full((6, 20, 20), 0.25)
    ref = _ref(u)
    alt = SimpleNamespace(energy=100.05)
    say = lambda *a: None
    compare_frame(_layers(u), ref.b, 100.05, ref, say=say, alt=alt)
    with pytest.raises(AssertionError):
        compare_frame(_layers(u), ref.b, 100.05, ref, say=say)
    with pytest.raises(AssertionError):
        compare_frame(_layers(u), ref.b, 100.2, ref, say=say, alt=alt)
