"""Batched clips of uneven size and the launch-shape autotuners, through the C ABI.

A batch runs the same kernel bodies as single clips with the same per-clip
workgroup layout and reduction order, in either launch layout (one launch over
all clips, or one per K), so its results must equal per-clip runs bitwise; the first frames are also checked against the FP64 oracle at the
parity bar (layers 1e-3 absolute, energy 1e-4 relative)."""
import os
import sys
import tempfile

import numpy as np
import pytest

import oracle as O
from parity import compare_frame
from scenes import make_clip

pytestmark = pytest.mark.gpu

P = O.default_params(state_precision="f32")


def _check_first_frame(L, b, e, c, label):
    """First frame of clip c against the oracle (3x8 schedule), as in the single-clip tests."""
    ref = O.decompose_clip(c.frames, c.ids, c.b_init, P, 3, 8, temporal=True, nframes=1, keep_starts=True)[0]
    alt = O.decompose_clip(c.frames, c.ids, c.b_init, O.default_params(), 3, 8, temporal=True, nframes=1)[0]
    return compare_frame(L, b, e, ref, 8, label, _say, alt)


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


def _clips():
    # (W, H, K, frames, seed): uneven sizes, K and lengths, ragged tiles
    spec = [(96, 64, 4, 3, 401), (160, 120, 6, 2, 402), (70, 45, 5, 4, 403), (130, 72, 8, 3, 404)]
    return [make_clip(W, H, K, F, s) for (W, H, K, F, s) in spec]


def _solver(c, **kw):
    import paper_1908_01961_amd as G
    s = G.Solver(c.width, c.height, G.default_params(c.K, gn_iters=3, pcg_iters=8, temporal=1, **kw))
    s.set_base_colors(c.b_init)
    return s


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _single_runs(torch, clips):
    out_all = []
    for c in clips:
        s = _solver(c)
        out = []
        lay = torch.empty((c.K + 4, c.height, c.width), dtype=torch.float32, device="cuda")
        for t in range(c.nframes):
            _, st = s.decompose_frame(_dev(torch, c.frames[t]), _dev(torch, c.ids[t]), lay)
            out.append((lay.cpu().numpy().copy(), st["energy_final"]))
        s.close()
        out_all.append(out)
    return out_all


def _batch_equals(torch, clips, single, launch):
    import paper_1908_01961_amd as G
    solvers = [_solver(c) for c in clips]
    batch = G.Batch(solvers)
    batch.set_launch(launch)
    assert batch.launch == launch
    lays = [torch.empty((c.K + 4, c.height, c.width), dtype=torch.float32, device="cuda") for c in clips]
    for t in range(max(c.nframes for c in clips)):
        frames = [_dev(torch, c.frames[t]) if t < c.nframes else None for c in clips]
        ids = [_dev(torch, c.ids[t]) if t < c.nframes else None for c in clips]
        e = batch.step(frames, ids, lays)
        for i, c in enumerate(clips):
            if t >= c.nframes:
                assert np.isnan(e[i])
                continue
            assert np.array_equal(lays[i].cpu().numpy(), single[i][t][0]), (launch, i, t)
            assert e[i] == single[i][t][1], (launch, i, t)
    batch.close()
    for s in solvers:
        s.close()


def test_one_launch_across_K_families_bitwise(torch):
    """K = 2, 9 and 13 in one batch: the one-launch layout takes the family
    bounded by 16 (every body up to K = 16 in one kernel); both layouts equal the
    single-clip runs bit for bit."""
    clips = [make_clip(W, H, K, F, s) for (W, H, K, F, s) in
             [(70, 40, 2, 2, 431), (96, 36, 9, 3, 432), (64, 50, 13, 2, 433)]]
    _say("batch across K families:", [(c.width, c.height, c.K, c.nframes) for c in clips])
    single = _single_runs(torch, clips)
    for launch in ("one", "per_k"):
        _batch_equals(torch, clips, single, launch)


def test_batch_launch_layout_calls(torch):
    """The layout switch refuses unknown layouts and pending steps; the tuner needs
    every clip's frame and then keeps one of the two layouts; a step after tuning
    still equals the single-clip run bit for bit."""
    import paper_1908_01961_amd as G
    clips = _clips()[:3]
    single = _single_runs(torch, clips)
    solvers = [_solver(c) for c in clips]
    batch = G.Batch(solvers)
    assert batch.launch == "one"                      # the default
    with pytest.raises(G.GidError) as e:
        batch.autotune()                              # no frame loaded yet
    assert e.value.status == 5
    assert solvers[0].lib.gid_batch_set_launch(batch.h, 7) == 1
    lays = [torch.empty((c.K + 4, c.height, c.width), dtype=torch.float32, device="cuda") for c in clips]
    batch.step_async([_dev(torch, c.frames[0]) for c in clips], [_dev(torch, c.ids[0]) for c in clips], lays)
    assert solvers[0].lib.gid_batch_set_launch(batch.h, 1) == 5   # a step is pending
    batch.synchronize()
    chosen = batch.autotune()
    assert chosen in ("one", "per_k") and batch.launch == chosen
    _say("batch tuner chose", chosen)
    e1 = batch.step([_dev(torch, c.frames[1]) for c in clips], [_dev(torch, c.ids[1]) for c in clips], lays)
    for i, c in enumerate(clips):
        assert np.array_equal(lays[i].cpu().numpy(), single[i][1][0]), i
        assert e1[i] == single[i][1][1], i
    batch.close()
    for s in solvers:
        s.close()


@pytest.mark.parametrize("launch", ["one", "per_k"])
def test_batch_equals_single_clips_bitwise(torch, launch):
    clips = _clips()
    _say("batch of", [(c.width, c.height, c.K, c.nframes) for c in clips], "launch", launch)
    _batch_equals(torch, clips, _single_runs(torch, clips), launch)


@pytest.mark.parametrize("launch", ["one", "per_k"])
def test_batch_of_one_K_splits_into_launches_bitwise(torch, launch):
    """Eleven clips of one K: per K, a step issues two launches (eight clips, then
    three); in one launch all eleven share the grid.  Clips that end early change
    the active set and the temporal flags between steps.  Every clip equals its
    single-clip run bit for bit."""
    sizes = [(40, 24), (64, 16), (72, 40), (48, 48), (96, 20), (33, 17), (64, 64), (80, 36),
             (56, 30), (100, 12), (45, 45)]
    clips = [make_clip(W, H, 4, 2 + (j % 3), 420 + j) for j, (W, H) in enumerate(sizes)]
    _say("batch of one K:", [(c.width, c.height, c.nframes) for c in clips], "launch", launch)
    _batch_equals(torch, clips, _single_runs(torch, clips), launch)


def test_batch_first_frames_match_oracle(torch):
    import paper_1908_01961_amd as G
    clips = _clips()
    solvers = [_solver(c) for c in clips]
    batch = G.Batch(solvers)
    lays = [torch.empty((c.K + 4, c.height, c.width), dtype=torch.float32, device="cuda") for c in clips]
    e = batch.step([_dev(torch, c.frames[0]) for c in clips], [_dev(torch, c.ids[0]) for c in clips], lays)
    for i, c in enumerate(clips):
        _, b = solvers[i].get_state()
        _check_first_frame(lays[i].cpu().numpy().astype(np.float64), b, e[i], c, f"batch clip {i}:")
    batch.close()


def test_batch_first_frames_match_oracle_at_mixed_sizes(torch):
    """The clip sizes of the uneven batch (320x240 ... 1280x720, K from the
    batch recipe), first frames, at the default launch shape: at 1280x720 a
    clip's 3600 tiles share at most 2048 workgroups."""
    import paper_1908_01961_amd as G
    from scenes import mixed_batch_specs
    specs = mixed_batch_specs(16, 400)[:8]
    clips = [make_clip(sp["width"], sp["height"], sp["K"], 1, sp["seed"]) for sp in specs]
    _say("batch first frames at the mixed sizes:", [(c.width, c.height, c.K) for c in clips])
    solvers = [_solver(c) for c in clips]
    batch = G.Batch(solvers)
    lays = [torch.empty((c.K + 4, c.height, c.width), dtype=torch.float32, device="cuda") for c in clips]
    e = batch.step([_dev(torch, c.frames[0]) for c in clips], [_dev(torch, c.ids[0]) for c in clips], lays)
    for i, c in enumerate(clips):
        _, b = solvers[i].get_state()
        _check_first_frame(lays[i].cpu().numpy().astype(np.float64), b, e[i], c,
                           f"mixed batch clip {i} ({c.width}x{c.height} K={c.K}):")
    batch.close()
    for s in solvers:
        s.close()


def test_batch_rejects_a_bad_frame_and_keeps_that_clip(torch):
    import paper_1908_01961_amd as G
    clips = _clips()[:2]
    solvers = [_solver(c) for c in clips]
    batch = G.Batch(solvers)
    batch.step([_dev(torch, c.frames[0]) for c in clips], [_dev(torch, c.ids[0]) for c in clips])
    u_before, _ = solvers[0].get_state()
    bad = clips[0].frames[1].copy()
    bad[0, 1, 1] = np.inf
    with pytest.raises(G.GidError) as ei:
        batch.step([_dev(torch, bad), _dev(torch, clips[1].frames[1])],
                   [_dev(torch, clips[0].ids[1]), _dev(torch, clips[1].ids[1])])
    assert ei.value.status == 4
    u_after, _ = solvers[0].get_state()
    assert torch.equal(u_before, u_after)
    batch.close()


def test_autotune_chooses_and_caches_a_launch_shape(torch):
    import paper_1908_01961_amd as G
    c = make_clip(320, 240, 4, 1, 405)
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "tune.txt")
        s = _solver(c)
        with pytest.raises(G.GidError) as e:          # the tuner times the real kernels on a loaded frame
            s.autotune(path)
        assert e.value.status == 5
        s.load_frame(_dev(torch, c.frames[0]), _dev(torch, c.ids[0]))
        n1 = s.autotune(path)
        assert 8 <= n1 <= 2048 and n1 % 8 == 0
        s2 = _solver(c)
        assert s2.autotune(path) == n1                 # read back from the cache
        assert open(path).read().split() == ["320", "240", "4", str(n1)]
        # a solve with the tuned shape still meets the bar
        lay = torch.empty((c.K + 4, c.height, c.width), dtype=torch.float32, device="cuda")
        b, st = s2.decompose_frame(_dev(torch, c.frames[0]), _dev(torch, c.ids[0]), lay)
        _check_first_frame(lay.cpu().numpy().astype(np.float64), b, st["energy_final"], c, "tuned launch:")
        s.close()
        s2.close()


@pytest.mark.parametrize("nb,expect", [(8, 8), (40, 40), (2048, 64)])
def test_few_workgroups_cover_every_tile(torch, nb, expect):
    """Fewer workgroups than tiles: every XCD owns a band of tiles that its
    workgroups take round-robin.  200 x 60 is 4 x 15 tiles of 64 x 4 (ragged right
    edge), bands of 7 or 8 tiles: 8 workgroups walk a whole band each, 40 share a
    band five ways, and a request above the tile count is clamped to it (64)."""
    c = make_clip(200, 60, 5, 1, 406)
    s = _solver(c)
    s.set_workgroups(nb)
    assert s.workgroups == expect
    lay = torch.empty((c.K + 4, c.height, c.width), dtype=torch.float32, device="cuda")
    b, st = s.decompose_frame(_dev(torch, c.frames[0]), _dev(torch, c.ids[0]), lay)
    _check_first_frame(lay.cpu().numpy().astype(np.float64), b, st["energy_final"], c, f"{nb} workgroups:")
    s.close()
