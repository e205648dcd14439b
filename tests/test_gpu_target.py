"""Energy-target continuation and frame-status rules of the single-clip solver,
through the C ABI.

With an energy target the schedule runs up to max_gn outer iterations and the
device skips the rest of a frame once its energy (Sec. 6, evaluated after every
outer iteration) is at or below the target.  The iterations it runs are the
fixed schedule's own, so a frame stopped after g iterations equals the fixed
g-iteration schedule bit for bit, and an unreachable target equals the fixed
max_gn schedule.  The oracle's per-iteration energies fix where a target
between two of them stops the frame.
"""
import sys

import numpy as np
import pytest

import oracle as O
from parity import compare_frame
from scenes import make_clip

pytestmark = pytest.mark.gpu


def _say(*msg):
    print("[gpu-case]", *msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    if not _t.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1908_01961_amd as G
    G.load_library()
    return _t


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _run(torch, c, G_, nframes, target=None, max_gn=0, use_graph=1, first_gn=None):
    import paper_1908_01961_amd as G
    s = G.Solver(c.width, c.height, G.default_params(c.K, gn_iters=G_, pcg_iters=8, temporal=1,
                                                     record_energy=0, use_graph=use_graph))
    s.set_base_colors(c.b_init)
    if first_gn is not None:
        s.set_energy_check_from(first_gn)
    out = []
    layers = torch.empty((c.K + 4, c.height, c.width), dtype=torch.float32, device="cuda")
    for t in range(nframes):
        if target is not None:
            s.set_energy_target(target[t] if hasattr(target, "__len__") else target, max_gn)
        b, st = s.decompose_frame(_dev(torch, c.frames[t]), _dev(torch, c.ids[t]), layers)
        out.append(dict(layers=layers.cpu().numpy().copy(), b=b, stats=st))
    s.close()
    return out


def test_unreachable_target_equals_the_fixed_schedule(torch):
    _say("energy target 1e-300 (unreachable), 160x120 K=6, 3 frames, max_gn 3 vs fixed 3x8")
    c = make_clip(160, 120, 6, 3, 201)
    for graph in (1, 0):
        fixed = _run(torch, c, 3, 3, use_graph=graph)
        tgt = _run(torch, c, 3, 3, target=1e-300, max_gn=3, use_graph=graph)
        for f, t in zip(fixed, tgt):
            assert np.array_equal(f["layers"], t["layers"])
            assert np.array_equal(f["b"], t["b"])
            assert t["stats"]["gn_done"] == 3 and len(t["stats"]["energy_half"]) == 3
            assert t["stats"]["energy_final"] == f["stats"]["energy_final"]
            assert t["stats"]["energy_half"][-1] == f["stats"]["energy_final"]


def test_reached_target_stops_after_the_first_iteration(torch):
    _say("energy target 1e300 (always met), 160x120 K=6, 3 frames, max_gn 5 vs fixed 1x8")
    c = make_clip(160, 120, 6, 3, 202)
    one = _run(torch, c, 1, 3)
    tgt = _run(torch, c, 3, 3, target=1e300, max_gn=5)
    for o, t in zip(one, tgt):
        assert t["stats"]["gn_done"] == 1
        assert np.array_equal(o["layers"], t["layers"])
        assert np.array_equal(o["b"], t["b"])
        assert t["stats"]["energy_final"] == o["stats"]["energy_final"]


def test_target_between_iterations_stops_where_the_oracle_says(torch):
    """Target halfway between the oracle's energies after outer iterations 2 and
    3 of the first frame: the GPU runs exactly three, and its frame matches the
    oracle's 3 x 8 schedule; a target halfway between iterations 1 and 2 stops
    after two."""
    _say("energy target between oracle iterations, 96x64 K=4 first frame, max_gn 6")
    c = make_clip(96, 64, 4, 1, 203)
    p = O.default_params(state_precision="f32")
    ref = O.decompose_clip(c.frames, c.ids, c.b_init, p, 4, 8, temporal=False, nframes=1, keep_starts=True)[0]
    E = [e for lab, e in ref.energies if lab == "B"]       # after each outer iteration
    assert E[0] > E[1] > E[2]
    for stop, tgt in ((3, 0.5 * (E[1] + E[2])), (2, 0.5 * (E[0] + E[1]))):
        g = _run(torch, c, 3, 1, target=tgt, max_gn=6)[0]
        assert g["stats"]["gn_done"] == stop, (stop, g["stats"]["energy_half"], E)
        for a, b in zip(g["stats"]["energy_half"], E):
            assert a == pytest.approx(b, rel=1e-4)
        ref_g = O.decompose_clip(c.frames, c.ids, c.b_init, p, stop, 8, temporal=False, nframes=1,
                                 keep_starts=True)[0]
        compare_frame(g["layers"], g["b"], g["stats"]["energy_final"], ref_g, 8, f"target stop {stop}:", _say)


def test_second_frame_before_synchronize_is_refused(torch):
    import paper_1908_01961_amd as G
    _say("pending-frame refusal, 64x48 K=3")
    c = make_clip(64, 48, 3, 3, 204)
    s = G.Solver(c.width, c.height, G.default_params(c.K, gn_iters=2, pcg_iters=4))
    s.set_base_colors(c.b_init)
    s.decompose_frame_async(_dev(torch, c.frames[0]), _dev(torch, c.ids[0]))
    with pytest.raises(G.GidError) as e:
        s.decompose_frame_async(_dev(torch, c.frames[1]), _dev(torch, c.ids[1]))
    assert e.value.status == 5
    with pytest.raises(G.GidError) as e:
        s.set_energy_target(1.0, 2)
    assert e.value.status == 5
    _, st = s.synchronize()
    assert st["frame_index"] == 0
    # a rejected frame between two good ones: its status reaches the caller and
    # the next frame continues from the first
    bad = c.frames[1].copy()
    bad[0, 3, 5] = np.nan
    s.decompose_frame_async(_dev(torch, bad), _dev(torch, c.ids[1]))
    with pytest.raises(G.GidError) as e:
        s.synchronize()
    assert e.value.status == 4
    _, st = s.decompose_frame(_dev(torch, c.frames[1]), _dev(torch, c.ids[1]))
    assert st["frame_index"] == 1 and np.isfinite(st["energy_final"])
    s.close()


@pytest.mark.parametrize("graph", [1, 0])
def test_checks_from_a_later_iteration(torch, graph):
    """Checks from outer iteration 3: an always-met target stops after iteration 3
    (the fixed 3-iteration schedule bit for bit, energies of iterations 1-2 NaN);
    with max_gn 2 below the first check the last iteration is still checked; an
    unreachable target runs max_gn as before."""
    _say("checks from iteration 3, 160x120 K=6, 2 frames, graph", graph)
    c = make_clip(160, 120, 6, 2, 203)
    three = _run(torch, c, 3, 2, use_graph=graph)
    two = _run(torch, c, 2, 2, use_graph=graph)
    met = _run(torch, c, 3, 2, target=1e300, max_gn=5, use_graph=graph, first_gn=3)
    short = _run(torch, c, 3, 2, target=1e300, max_gn=2, use_graph=graph, first_gn=3)
    never = _run(torch, c, 3, 2, target=1e-300, max_gn=4, use_graph=graph, first_gn=3)
    four = _run(torch, c, 4, 2, use_graph=graph)
    for f3, f2, f4, m, sh, nv in zip(three, two, four, met, short, never):
        assert m["stats"]["gn_done"] == 3
        assert np.array_equal(f3["layers"], m["layers"]) and np.array_equal(f3["b"], m["b"])
        assert m["stats"]["energy_final"] == f3["stats"]["energy_final"]
        eh = m["stats"]["energy_half"]
        assert len(eh) == 3 and np.isnan(eh[0]) and np.isnan(eh[1]) and eh[2] == f3["stats"]["energy_final"]
        assert sh["stats"]["gn_done"] == 2
        assert np.array_equal(f2["layers"], sh["layers"])
        assert sh["stats"]["energy_final"] == f2["stats"]["energy_final"]
        assert not np.isnan(sh["stats"]["energy_half"][-1])
        assert nv["stats"]["gn_done"] == 4
        assert np.array_equal(f4["layers"], nv["layers"])
        assert nv["stats"]["energy_final"] == f4["stats"]["energy_final"]


def test_check_from_refuses_bad_values(torch):
    import paper_1908_01961_amd as G
    c = make_clip(64, 48, 4, 1, 204)
    s = G.Solver(c.width, c.height, G.default_params(c.K))
    for bad in (0, 65):
        with pytest.raises(G.GidError) as e:
            s.set_energy_check_from(bad)
        assert e.value.status == 1
    s.set_energy_check_from(2)
    s.close()
