"""The schedule comparison used by the GPU tests, checked on the CPU with
constructed inputs (no GPU, no solver)."""
from types import SimpleNamespace

import numpy as np
import pytest

from parity import BRANCH_EPS, LOOSE_BOUND, TOL_LAYER, compare_frame, nearest_branch_value


def _ref(u, starts=()):
    return SimpleNamespace(u=u, b=np.full((2, 3), 0.4), energy=100.0, starts=list(starts))


def _layers(u):
    return np.concatenate([np.exp(u[:3]), u[3:]])


def _starts(u, n=3):
    return [u.copy() for _ in range(n)]


def test_nearest_branch_value_looks_at_the_neighbourhood_after_step_0():
    st = [np.full((6, 5, 5), 0.5) for _ in range(3)]
    st[0][4, 2, 2] = 1e-12          # the given start state is not a branch point of the schedule
    st[2][5, 2, 3] = -3e-9          # right neighbour, last step
    st[1][3, 0, 0] = 1e-10          # far away
    st[1][1, 2, 2] = 0.0            # r plane: no branch
    assert nearest_branch_value(st, 2, 2) == pytest.approx(3e-9)
    assert nearest_branch_value(st, 4, 4) == 0.5
    assert nearest_branch_value(st, 4, 1, radius=2) == 0.5          # every traced value is 4+ steps away
    assert nearest_branch_value(st, 2, 1, radius=2) == pytest.approx(3e-9)
    assert nearest_branch_value(st, 1, 1, radius=2) == pytest.approx(1e-10)


def test_elements_over_the_bar_must_sit_at_branch_points():
    H, W, n = 40, 40, 6
    u = np.full((n, H, W), 0.25)
    st = _starts(u)
    st[1][4, 10, 10] = -2e-9                      # a branch point traced by the oracle
    ref = _ref(u, st)
    say = lambda *a: None
    L = _layers(u)
    rep = compare_frame(L, ref.b, 100.0, ref, say=say)
    assert rep["n_over"] == 0 and rep["flips"] == 0
    ok = L.copy()
    ok[4, 10, 10] += 2e-2                         # at the branch point
    ok[5, 10, 11] += 4e-3                         # its neighbour
    ok[3, 12, 10] += 2e-3                         # two steps away
    rep = compare_frame(ok, ref.b, 100.0, ref, say=say)
    assert rep["n_over"] == 3 and rep["flips"] == 3 and rep["off_branch"] == []
    # one injected error away from any branch point fails, however small the count
    bad = ok.copy()
    bad[4, 30, 30] += 2 * TOL_LAYER
    with pytest.raises(AssertionError):
        compare_frame(bad, ref.b, 100.0, ref, say=say)
    # a traced value that is not within rounding distance of zero is no branch point
    st2 = _starts(u)
    st2[1][4, 10, 10] = 10 * BRANCH_EPS
    with pytest.raises(AssertionError):
        compare_frame(ok, ref.b, 100.0, _ref(u, st2), say=say)
    # no trajectory: nothing may exceed the bar
    with pytest.raises(AssertionError):
        compare_frame(ok, ref.b, 100.0, _ref(u), say=say)
    worse = ok.copy()
    worse[4, 10, 10] += 2 * LOOSE_BOUND           # at the branch point, beyond the loose bound
    with pytest.raises(AssertionError):
        compare_frame(worse, ref.b, 100.0, ref, say=say)


def test_layers_energy_and_colours_bars():
    u = np.full((6, 20, 20), 0.25)
    ref = _ref(u, _starts(u))
    say = lambda *a: None
    L = _layers(u)
    with pytest.raises(AssertionError):         # reflectance layers are compared as R = exp(r)
        r = L.copy()
        r[0, 1:4, 1:4] *= 1.01
        compare_frame(r, ref.b, 100.0, ref, say=say)
    with pytest.raises(AssertionError):         # energy bar
        compare_frame(L, ref.b, 100.02, ref, say=say)
    with pytest.raises(AssertionError):         # colour bar
        compare_frame(L, ref.b + 2e-3, 100.0, ref, say=say)


def test_fp64_storage_energy_is_accepted_only_with_branch_flips():
    u = np.full((6, 20, 20), 0.25)
    st = _starts(u)
    st[2][4, 5, 5] = 1e-10
    ref = _ref(u, st)
    alt = SimpleNamespace(energy=100.05)
    say = lambda *a: None
    L = _layers(u)
    with pytest.raises(AssertionError):          # no flip: the FP32-storage oracle decides
        compare_frame(L, ref.b, 100.05, ref, say=say, alt=alt)
    split = L.copy()
    split[4, 5, 5] += 1e-2
    rep = compare_frame(split, ref.b, 100.05, ref, say=say, alt=alt)
    assert rep["flips"] == 1
    with pytest.raises(AssertionError):
        compare_frame(split, ref.b, 100.2, ref, say=say, alt=alt)
