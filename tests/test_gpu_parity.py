"""GPU path versus the FP64 oracle, through the C ABI (libgid via the binding).

Tolerances: single kernels fed the same FP32 state are compared with the
oracle evaluated at that state (FP32 per-pixel arithmetic against FP64: 1e-5 of
the plane's largest magnitude; FP64 sums and energies: 1e-9 relative).  Single
Gauss-Newton steps fed the oracle's state at full frame sizes: layers within
1e-3.  Whole schedules (fixed G x P, same inputs): layers within 1e-3 absolute,
colours within 1e-3 and the final energy within 1e-4 relative, with the
rounding-decided branch points of the non-negativity reweighting handled as
described in tests/parity.py.

Every oracle input is synthetic or the oracle's own output; GPU results only
ever appear on the compared side.
"""
import math
import sys
from dataclasses import replace

import numpy as np
import pytest

import oracle as O
from oracle.basecolor import bstep, bstep_sums
from oracle.energy import chromaticity, energy_terms, prepare_frame
from oracle.gauss_newton import apply_normal, jacobi_diag, linearise, rhs
from oracle.gauss_newton import pcg
from oracle.schedule import init_state, store
from parity import compare_frame
from scenes import downsample_clip, make_clip, workload_clip

pytestmark = pytest.mark.gpu

TERMS = ("data", "cluster", "rsparsity", "rconsist", "mono", "isparsity", "smooth", "nonneg")
P = O.default_params()
# Schedules are compared with the oracle storing its unknowns in FP32 where the
# GPU stores them (all oracle arithmetic stays FP64), so both sides start every
# step from equally rounded states.
P32 = O.default_params(state_precision="f32")


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


def _solver(torch, W, H, K, **kw):
    import paper_1908_01961_amd as G
    prm = G.default_params(K, **kw)
    return G.Solver(W, H, prm)


def _dev(torch, a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def _u_np(u):
    return u.detach().cpu().numpy().astype(np.float64)


def _rel(a, b):
    return float(np.abs(a - b).max() / max(1e-30, np.abs(b).max()))


# --------------------------------------------------------------- single steps

@pytest.fixture(scope="module")
def step_case(torch):
    """A 70x45 video frame pair (ragged tiles), K = 5, temporal prior on.  The
    oracle decomposes frame 0; its result (rounded to FP32), perturbed, is the
    state both sides evaluate frame 1 at."""
    _say("step_case 70x45 K=5 seed 61")
    c = make_clip(70, 45, 5, 2, 61)
    f0 = O.decompose_clip(c.frames, c.ids, c.b_init, P32, 3, 8, temporal=True, nframes=1)[0]
    prev_r = f0.u[:3].astype(np.float32)
    b0 = f0.b.copy()
    rng = np.random.default_rng(5)
    u32 = (f0.u + 0.02 * rng.standard_normal(f0.u.shape)).astype(np.float32)
    s = _solver(torch, 70, 45, 5, temporal=1)
    s.set_base_colors(c.b_init)
    s.set_prev_frame(_dev(torch, c.frames[0]), _dev(torch, prev_r))
    s.load_frame(_dev(torch, c.frames[1]), _dev(torch, c.ids[1]))
    u_t = _dev(torch, u32)
    s.set_state(u_t, b0)
    prev_C = chromaticity(c.frames[0].astype(np.float64), P)
    fd = prepare_frame(c.frames[1], c.ids[1], P, prev_C, prev_r.astype(np.float64))
    return dict(c=c, s=s, u=u32.astype(np.float64), b=b0, fd=fd, u_t=u_t)


def test_energy_single_step(step_case):
    s, u, b, fd = step_case["s"], step_case["u"], step_case["b"], step_case["fd"]
    E, terms = s.eval_energy()
    ref = energy_terms(u, b, fd, P)
    for k in TERMS:
        assert terms[k] == pytest.approx(ref[k], rel=1e-9, abs=1e-9), k
    assert E == pytest.approx(sum(ref.values()), rel=1e-9)


def test_rhs_and_diag_single_step(step_case):
    s, u, b, fd = step_case["s"], step_case["u"], step_case["b"], step_case["fd"]
    g, d = s.eval_rhs()
    lin = linearise(u, b, fd, P)
    g_ref, d_ref = rhs(lin), jacobi_diag(lin)
    g, d = _u_np(g), _u_np(d)
    for v in range(u.shape[0]):
        assert _rel(g[v], g_ref[v]) < 1e-5, ("g", v, _rel(g[v], g_ref[v]))
        assert _rel(d[v], d_ref[v]) < 1e-5, ("diag", v)


def test_apply_normal_single_step(torch, step_case):
    s, u, b, fd = step_case["s"], step_case["u"], step_case["b"], step_case["fd"]
    rng = np.random.default_rng(7)
    p = rng.standard_normal(u.shape).astype(np.float32)
    q = _u_np(s.apply_normal(_dev(torch, p)))
    q_ref = apply_normal(p.astype(np.float64), linearise(u, b, fd, P))
    for v in range(u.shape[0]):
        assert _rel(q[v], q_ref[v]) < 1e-5, ("q", v, _rel(q[v], q_ref[v]))


def test_bstep_sums_single_step(step_case):
    s, u, b, fd = step_case["s"], step_case["u"], step_case["b"], step_case["fd"]
    A, h = s.bstep_sums()
    A_ref, h_ref = bstep_sums(u, b, fd.I, P)
    assert _rel(A, A_ref) < 1e-9 and _rel(h, h_ref) < 1e-9


def test_base_step_single_step(torch, step_case):
    s, u, b, fd, c = step_case["s"], step_case["u"], step_case["b"], step_case["fd"], step_case["c"]
    s.set_state(step_case["u_t"], b)
    ok = s.base_step()
    _, b_gpu = s.get_state()
    b_ref, ok_ref = bstep(u, b, c.b_init, fd.I, P)
    assert ok == ok_ref
    assert np.abs(b_gpu - b_ref).max() < 1e-9
    s.set_state(step_case["u_t"], b)


def test_layer_step_single_step(torch, step_case):
    s, u, b, fd = step_case["s"], step_case["u"], step_case["b"], step_case["fd"]
    s.set_state(step_case["u_t"], b)
    rz = s.layer_step()
    u_gpu, _ = s.get_state()
    lin = linearise(u, b, fd, P)
    d, info = O.pcg(lin, 8)
    un = u + d
    assert np.abs(_u_np(u_gpu) - un).max() < 1e-4
    assert rz == pytest.approx(info["rz"], rel=1e-3)
    s.set_state(step_case["u_t"], b)


# ------------------------------------------- single GN steps at full frame size

def _gn_steps_anchored(torch, clip, frames, G_, P_, K):
    """For each listed frame, run the oracle's schedule (its own chain before
    it) and, at every Gauss-Newton step, give the GPU the oracle's state at the
    start of the step and compare the GPU's layer step with the oracle's."""
    W, H = clip.width, clip.height
    last = max(frames)
    chain = O.decompose_clip(clip.frames, clip.ids, clip.b_init, P32, G_, P_, temporal=True, nframes=last)
    s = _solver(torch, W, H, K, gn_iters=G_, pcg_iters=P_, temporal=1)
    s.set_base_colors(clip.b_init)
    worst = 0.0
    for t in frames:
        if t == 0:
            fd = prepare_frame(clip.frames[0], clip.ids[0], P32, None, None)
            u = store(init_state(fd.I, fd.ids, clip.b_init), P32)
            b = np.asarray(clip.b_init, np.float64).copy()
            s.reset_clip()
        else:
            prev = chain[t - 1]
            r_prev = prev.u[:3].astype(np.float32)
            fd = prepare_frame(clip.frames[t], clip.ids[t], P32, prev.fd.C, r_prev.astype(np.float64))
            u, b = prev.u.astype(np.float32).astype(np.float64), prev.b.copy()
            s.set_prev_frame(_dev(torch, clip.frames[t - 1]), _dev(torch, r_prev))
        s.load_frame(_dev(torch, clip.frames[t]), _dev(torch, clip.ids[t]))
        for g in range(G_):
            s.set_state(_dev(torch, u.astype(np.float32)), b)
            s.layer_step()
            ug = _u_np(s.get_state()[0])
            d, _ = pcg(linearise(u, b, fd, P32), P_)
            un = store(u + d, P32)
            err = float(np.abs(ug - un).max())
            worst = max(worst, err)
            _say(f"  frame {t} GN step {g}: max |gpu - oracle| {err:.2e} over {un.size} values")
            assert err <= 1e-3, (t, g, err)
            u = un
            b, _ = bstep(u, b, clip.b_init, fd.I, P32)
    s.close()
    return worst


def test_gn_steps_anchored_640x480_full_size(torch):
    _say("GN steps anchored to the oracle, video_640x480_k6 frames 0 and 2, 3x8")
    _gn_steps_anchored(torch, workload_clip("video_640x480_k6", nframes=3), [0, 2], 3, 8, 6)


def test_gn_steps_anchored_1280x720_full_size(torch):
    _say("GN steps anchored to the oracle, video_1280x720_k8 frame 0, 3x8")
    _gn_steps_anchored(torch, workload_clip("video_1280x720_k8", nframes=1), [0], 3, 8, 8)


def test_gn_steps_anchored_1920x1080_full_size(torch):
    _say("GN steps anchored to the oracle, video_1920x1080_k10 frame 0, first 2 GN steps of 3x8")
    _gn_steps_anchored(torch, workload_clip("video_1920x1080_k10", nframes=1), [0], 2, 8, 10)


# -------------------------------------------------------------- whole schedules

def _run_gpu_clip(torch, clip, G_, P_, nframes, temporal, refine="every", **kw):
    s = _solver(torch, clip.width, clip.height, clip.K, gn_iters=G_, pcg_iters=P_, temporal=int(temporal),
                refine_mode=refine, record_energy=1, **kw)
    s.set_base_colors(clip.b_init)
    out = []
    layers = torch.empty((clip.K + 4, clip.height, clip.width), dtype=torch.float32, device="cuda")
    for t in range(nframes):
        b, st = s.decompose_frame(_dev(torch, clip.frames[t]), _dev(torch, clip.ids[t]), layers)
        u, _ = s.get_state()
        out.append(dict(layers=_u_np(layers), u=_u_np(u), b=b, stats=st))
    s.close()
    return out


def _compare(gpu, orc, P_, label="", alt=None):
    alt = alt or [None] * len(orc)
    return [compare_frame(g["layers"], g["b"], g["stats"]["energy_final"], o, P_, f"{label} frame {t}:", _say, a)
            for t, (g, o, a) in enumerate(zip(gpu, orc, alt))]


def _oracle_clip(c, G_, P_, nframes=None, temporal=True, p=P32, **kw):
    return O.decompose_clip(c.frames, c.ids, c.b_init, p, G_, P_, temporal=temporal, nframes=nframes,
                            keep_starts=True, **kw)


def _oracle_clip64(c, G_, P_, nframes=None, temporal=True, p=P32, **kw):
    """The same run with the unknowns stored in FP64 (energy reference only)."""
    return O.decompose_clip(c.frames, c.ids, c.b_init, replace(p, state_precision="f64"), G_, P_,
                            temporal=temporal, nframes=nframes, **kw)


def test_schedule_single_frame_64x48(torch):
    _say("schedule single_64x48_k4 5x10")
    c = workload_clip("single_64x48_k4")
    gpu = _run_gpu_clip(torch, c, 5, 10, 1, False)
    orc = _oracle_clip(c, 5, 10, temporal=False)
    rep = _compare(gpu, orc, 10)
    assert rep[0]["n_over"] == 0                                       # every element within the bar
    eh = gpu[0]["stats"]["energy_half"]
    assert len(eh) == 10
    for a, (_, b) in zip(eh, orc[0].energies):
        assert a == pytest.approx(b, rel=1e-4)


def _anchored(torch, clip, G_, P_, nframes, check=None, **okw):
    """Video parity frame by frame: the oracle runs its own chain; for every
    frame t >= 1 (or the frames in `check`) the GPU is loaded with the oracle's
    frame t-1 result (rounded to FP32: the GPU's storage precision) and must
    reproduce the oracle's frame t, which the oracle recomputes from that same
    rounded state."""
    p = O.default_params(state_precision="f32", **okw)
    chain = O.decompose_clip(clip.frames, clip.ids, clip.b_init, p, G_, P_, temporal=True, nframes=nframes)
    s = _solver(torch, clip.width, clip.height, clip.K, gn_iters=G_, pcg_iters=P_, temporal=1, record_energy=1,
                **({"cr_mode": okw["cr_mode"]} if "cr_mode" in okw else {}))
    layers = torch.empty((clip.K + 4, clip.height, clip.width), dtype=torch.float32, device="cuda")
    reps = []
    for t in (check if check is not None else range(1, nframes)):
        prev = chain[t - 1]
        u32 = prev.u.astype(np.float32)
        s.set_base_colors(clip.b_init)
        s.set_prev_frame(_dev(torch, clip.frames[t - 1]), _dev(torch, u32[:3]))
        s.set_state(_dev(torch, u32), prev.b)
        b, st = s.decompose_frame(_dev(torch, clip.frames[t]), _dev(torch, clip.ids[t]), layers)
        kw = dict(u0=u32.astype(np.float64), prev=(prev.fd.C, u32[:3].astype(np.float64)))
        ref = O.decompose_frame(clip.frames[t], clip.ids[t], prev.b, clip.b_init, p, G_, P_, keep_starts=True, **kw)
        alt = O.decompose_frame(clip.frames[t], clip.ids[t], prev.b, clip.b_init, replace(p, state_precision="f64"),
                                G_, P_, **kw)
        reps.append(compare_frame(_u_np(layers), b, st["energy_final"], ref, P_, f"anchored frame {t}:", _say, alt))
    s.close()
    return reps


def test_video_anchored_160x120(torch):
    _say("anchored video 160x120 K=6, 6 frames, 3x8")
    _anchored(torch, make_clip(160, 120, 6, 6, 200), 3, 8, 6)


def test_video_anchored_640x480_full_size(torch):
    _say("anchored video_640x480_k6, first 3 frames (full size), 3x8")
    _anchored(torch, workload_clip("video_640x480_k6", nframes=3), 3, 8, 3)


def test_video_anchored_640x480_deep_in_the_clip(torch):
    _say("anchored video_640x480_k6, frames 10, 20 and 29 of 30 (full size), 3x8")
    _anchored(torch, workload_clip("video_640x480_k6", workers=8), 3, 8, 30, check=(10, 20, 29))


def test_video_anchored_1280x720_full_size(torch):
    _say("anchored video_1280x720_k8, frames 1 and 2 (full size), 3x8")
    _anchored(torch, workload_clip("video_1280x720_k8", nframes=3, workers=3), 3, 8, 3)


def test_video_anchored_1080p_downsampled_96x54(torch):
    _say("anchored 1920x1080 K=10 scene, 96x54 area-averaged copy, 5 frames")
    full = make_clip(1920, 1080, 10, 5, 500, amp=0.35, supersample=False)
    _anchored(torch, downsample_clip(full, 20), 3, 8, 5)


def test_video_free_running_first_frames(torch):
    """Free-running chains (both sides warm-start from their own results): the
    first frame meets the bar and the first two frames' energies agree within
    1e-4.  Later frames are covered by the anchored tests: a branch point taken
    differently on frame t changes the warm start of frame t+1."""
    for name, c in (("160x120 K=6", make_clip(160, 120, 6, 2, 200)),
                    ("640x480 K=6", workload_clip("video_640x480_k6", nframes=2))):
        _say("free-running", name, "2 frames 3x8")
        gpu = _run_gpu_clip(torch, c, 3, 8, 2, True)
        orc = _oracle_clip(c, 3, 8, nframes=2)
        alt = _oracle_clip64(c, 3, 8, nframes=2)
        _compare(gpu[:1], orc[:1], 8, name, alt[:1])
        for g, o, a in zip(gpu, orc, alt):
            e = g["stats"]["energy_final"]
            assert min(abs(e - o.energy) / o.energy, abs(e - a.energy) / a.energy) <= 1e-4


@pytest.mark.parametrize("W,H,K", [(2, 2, 2), (70, 45, 1), (33, 17, 16), (129, 9, 3)])
def test_schedule_edge_shapes(torch, W, H, K):
    _say(f"edge shape {W}x{H} K={K}")
    c = make_clip(W, H, K, 3, 900 + W + K)
    gpu = _run_gpu_clip(torch, c, 2, 6, 1, True)
    _compare(gpu, _oracle_clip(c, 2, 6, nframes=1), 6, alt=_oracle_clip64(c, 2, 6, nframes=1))
    _anchored(torch, c, 2, 6, 3)


def test_refine_modes_and_literal_cr(torch):
    _say("refine modes first/off and literal chromaticity term, 96x64 K=4 3 frames")
    c = make_clip(96, 64, 4, 3, 321)
    for mode in ("first", "off"):
        gpu = _run_gpu_clip(torch, c, 2, 8, 2, True, refine=mode)
        orc = _oracle_clip(c, 2, 8, nframes=2, refine_mode=mode)
        _compare(gpu[:1], orc[:1], 8, f"refine={mode}", _oracle_clip64(c, 2, 8, nframes=1, refine_mode=mode))
        # with refinement off after the first frame, the second frame's colours are the first's
        assert np.array_equal(gpu[1]["b"], gpu[0]["b"])
    pl = O.default_params(cr_mode="literal", state_precision="f32")
    gpu = _run_gpu_clip(torch, c, 2, 8, 1, True, cr_mode="literal")
    _compare(gpu, _oracle_clip(c, 2, 8, nframes=1, p=pl), 8, "literal CR", _oracle_clip64(c, 2, 8, nframes=1, p=pl))
    _anchored(torch, c, 2, 8, 3, cr_mode="literal")


def test_printed_pixel_sum_bstep_scale(torch):
    """The base-colour data sum taken as printed (bstep_scale "sum", Sec. 6.3):
    on the 64x48 K = 4 scene every base-colour step of a 3 x 10 schedule would
    drive a colour component below 1e-4 and is rejected, on both sides."""
    _say("bstep_scale=sum, single_64x48_k4 3x10")
    c = workload_clip("single_64x48_k4")
    ps = O.default_params(bstep_scale="sum", state_precision="f32")
    gpu = _run_gpu_clip(torch, c, 3, 10, 1, False, bstep_scale="sum")
    orc = _oracle_clip(c, 3, 10, temporal=False, p=ps)
    assert all(e_b == e_t for (_, e_t), (_, e_b) in zip(orc[0].energies[0::2], orc[0].energies[1::2]))
    assert gpu[0]["stats"]["bstep_rejected"] == 3
    assert np.array_equal(gpu[0]["b"], c.b_init)
    rep = _compare(gpu, orc, 10, "bstep_scale=sum")
    assert rep[0]["n_over"] == 0


# --------------------------------------------------- determinism, graph, resume

def test_graph_replay_matches_direct_launches_bitwise(torch):
    _say("graph vs direct launches, 128x96 K=6 4 frames")
    c = make_clip(128, 96, 6, 4, 77)
    a = _run_gpu_clip(torch, c, 3, 8, 4, True, use_graph=1)
    b = _run_gpu_clip(torch, c, 3, 8, 4, True, use_graph=0)
    a2 = _run_gpu_clip(torch, c, 3, 8, 4, True, use_graph=1)
    for x, y, z in zip(a, b, a2):
        assert np.array_equal(x["layers"], y["layers"]) and np.array_equal(x["layers"], z["layers"])
        assert x["stats"]["energy_final"] == y["stats"]["energy_final"] == z["stats"]["energy_final"]


def test_checkpoint_resume_is_bitwise(torch):
    _say("checkpoint / resume, 96x64 K=4 4 frames")
    c = make_clip(96, 64, 4, 4, 88)
    full = _run_gpu_clip(torch, c, 2, 6, 4, True)
    s = _solver(torch, 96, 64, 4, gn_iters=2, pcg_iters=6, record_energy=1)
    s.set_base_colors(c.b_init)
    for t in range(2):
        s.decompose_frame(_dev(torch, c.frames[t]), _dev(torch, c.ids[t]))
    blob = s.save_state()
    s.close()
    s2 = _solver(torch, 96, 64, 4, gn_iters=2, pcg_iters=6, record_energy=1)
    s2.load_state(blob)
    layers = torch.empty((8, 64, 96), dtype=torch.float32, device="cuda")
    for t in range(2, 4):
        b, st = s2.decompose_frame(_dev(torch, c.frames[t]), _dev(torch, c.ids[t]), layers)
        assert np.array_equal(_u_np(layers), full[t]["layers"])
        assert st["energy_final"] == full[t]["stats"]["energy_final"]


def test_bad_input_frame_is_rejected_and_state_kept(torch):
    _say("non-finite frame and out-of-range ids are rejected")
    import paper_1908_01961_amd as G
    c = make_clip(64, 32, 3, 3, 5)
    s = _solver(torch, 64, 32, 3, gn_iters=2, pcg_iters=4)
    s.set_base_colors(c.b_init)
    s.decompose_frame(_dev(torch, c.frames[0]), _dev(torch, c.ids[0]))
    u_before, b_before = s.get_state()
    bad = c.frames[1].copy()
    bad[1, 3, 4] = np.nan
    with pytest.raises(G.GidError) as ei:
        s.decompose_frame(_dev(torch, bad), _dev(torch, c.ids[1]))
    assert ei.value.status == 4
    ids_bad = c.ids[1].copy()
    ids_bad[0, 0] = 3
    with pytest.raises(G.GidError):
        s.decompose_frame(_dev(torch, c.frames[1]), _dev(torch, ids_bad))
    u_after, b_after = s.get_state()
    assert torch.equal(u_before, u_after) and np.array_equal(b_before, b_after)
    # the clip continues as if the bad frames had not been offered
    _, st = s.decompose_frame(_dev(torch, c.frames[1]), _dev(torch, c.ids[1]))
    assert st["frame_index"] == 1


def test_zero_operator_hits_pcg_breakdown_guard(torch):
    _say("zero operator -> PCG breakdown guard")
    zero = dict(lam_data=0.0, lam_cluster=0.0, lam_r_sparsity=0.0, lam_r_consistency=0.0,
                lam_monochrome=0.0, lam_i_sparsity=0.0, lam_smoothness=0.0, lam_non_neg=0.0)
    c = make_clip(64, 16, 2, 1, 3)
    s = _solver(torch, 64, 16, 2, gn_iters=1, pcg_iters=4, refine_mode="off", **zero)
    s.set_base_colors(c.b_init)
    s.load_frame(_dev(torch, c.frames[0]), _dev(torch, c.ids[0]))
    u0, _ = s.get_state()
    s.layer_step()
    u1, _ = s.get_state()
    assert torch.equal(u0, u1)
