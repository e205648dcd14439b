"""Spatial pairs of the consistency prior (Sec. 6.1, spatial_pairs = 1) on the
GPU against the oracle with the same reading, through the C ABI: single steps
at one FP32 state (energy terms to 1e-9, right-hand side, diagonal and the
normal-equation product to 1e-5 of the plane maximum), a whole schedule on a
single frame and anchored video frames (the schedule bar of tests/parity.py)."""
import sys
from dataclasses import replace

import numpy as np
import pytest

import oracle as O
from oracle.energy import chromaticity, energy_terms, prepare_frame
from oracle.gauss_newton import apply_normal, jacobi_diag, linearise, rhs
from parity import compare_frame
from scenes import make_clip, workload_clip

pytestmark = pytest.mark.gpu
PS = O.default_params(spatial_pairs=True)
PS32 = replace(PS, state_precision="f32")
TERMS = ("data", "cluster", "rsparsity", "rconsist", "mono", "isparsity", "smooth", "nonneg")


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


def _np(t):
    return t.detach().cpu().numpy().astype(np.float64)


def _rel(a, b):
    return float(np.abs(a - b).max() / max(1e-30, np.abs(b).max()))


@pytest.fixture(scope="module")
def case(torch):
    import paper_1908_01961_amd as G
    _say("spatial pairs single steps, 70x45 K=5 with the temporal prior")
    c = make_clip(70, 45, 5, 2, 62)
    f0 = O.decompose_clip(c.frames, c.ids, c.b_init, PS32, 3, 8, temporal=True, nframes=1)[0]
    prev_r = f0.u[:3].astype(np.float32)
    rng = np.random.default_rng(6)
    u32 = (f0.u + 0.02 * rng.standard_normal(f0.u.shape)).astype(np.float32)
    s = G.Solver(70, 45, G.default_params(5, temporal=1, spatial_pairs=1))
    s.set_base_colors(c.b_init)
    s.set_prev_frame(_dev(torch, c.frames[0]), _dev(torch, prev_r))
    s.load_frame(_dev(torch, c.frames[1]), _dev(torch, c.ids[1]))
    s.set_state(_dev(torch, u32), f0.b)
    fd = prepare_frame(c.frames[1], c.ids[1], PS, chromaticity(c.frames[0].astype(np.float64), PS),
                       prev_r.astype(np.float64))
    assert fd.sp_edges.sum() > 100
    yield dict(s=s, u=u32.astype(np.float64), b=f0.b, fd=fd)
    s.close()


def test_energy_with_spatial_pairs(case):
    s, u, b, fd = case["s"], case["u"], case["b"], case["fd"]
    E, terms = s.eval_energy()
    ref = energy_terms(u, b, fd, PS)
    for k in TERMS:
        assert terms[k] == pytest.approx(ref[k], rel=1e-9, abs=1e-9), k
    assert E == pytest.approx(sum(ref.values()), rel=1e-9)


def test_rhs_diag_and_product_with_spatial_pairs(torch, case):
    s, u, b, fd = case["s"], case["u"], case["b"], case["fd"]
    lin = linearise(u, b, fd, PS)
    g, d = s.eval_rhs()
    g, d = _np(g), _np(d)
    g_ref, d_ref = rhs(lin), jacobi_diag(lin)
    p = np.random.default_rng(8).standard_normal(u.shape).astype(np.float32)
    q = _np(s.apply_normal(_dev(torch, p)))
    q_ref = apply_normal(p.astype(np.float64), lin)
    for v in range(u.shape[0]):
        assert _rel(g[v], g_ref[v]) < 1e-5, ("g", v)
        assert _rel(d[v], d_ref[v]) < 1e-5, ("diag", v)
        assert _rel(q[v], q_ref[v]) < 1e-5, ("q", v)


def test_schedule_with_spatial_pairs(torch):
    import paper_1908_01961_amd as G
    _say("spatial pairs: 64x48 K=4 single frame 5x10, then anchored 160x120 K=6 frames 1-2 3x8")
    c = workload_clip("single_64x48_k4")
    s = G.Solver(c.width, c.height, G.default_params(c.K, gn_iters=5, pcg_iters=10, temporal=0, record_energy=1,
                                                     spatial_pairs=1))
    s.set_base_colors(c.b_init)
    layers = torch.empty((c.K + 4, c.height, c.width), dtype=torch.float32, device="cuda")
    b, st = s.decompose_frame(_dev(torch, c.frames[0]), _dev(torch, c.ids[0]), layers)
    s.close()
    ref = O.decompose_clip(c.frames, c.ids, c.b_init, PS32, 5, 10, temporal=False, keep_starts=True)[0]
    rep = compare_frame(_np(layers), b, st["energy_final"], ref, 10, "spatial 64x48:", _say)
    assert rep["n_over"] == 0
    # anchored video frames
    v = make_clip(160, 120, 6, 3, 205)
    chain = O.decompose_clip(v.frames, v.ids, v.b_init, PS32, 3, 8, temporal=True, nframes=3)
    s = G.Solver(v.width, v.height, G.default_params(v.K, gn_iters=3, pcg_iters=8, temporal=1, record_energy=1,
                                                     spatial_pairs=1))
    layers = torch.empty((v.K + 4, v.height, v.width), dtype=torch.float32, device="cuda")
    for t in (1, 2):
        prev = chain[t - 1]
        u32 = prev.u.astype(np.float32)
        s.set_base_colors(v.b_init)
        s.set_prev_frame(_dev(torch, v.frames[t - 1]), _dev(torch, u32[:3]))
        s.set_state(_dev(torch, u32), prev.b)
        b, st = s.decompose_frame(_dev(torch, v.frames[t]), _dev(torch, v.ids[t]), layers)
        kw = dict(u0=u32.astype(np.float64), prev=(prev.fd.C, u32[:3].astype(np.float64)))
        ref = O.decompose_frame(v.frames[t], v.ids[t], prev.b, v.b_init, PS32, 3, 8, keep_starts=True, **kw)
        alt = O.decompose_frame(v.frames[t], v.ids[t], prev.b, v.b_init, PS, 3, 8, **kw)
        compare_frame(_np(layers), b, st["energy_final"], ref, 8, f"spatial anchored frame {t}:", _say, alt)
    s.close()
