"""Base-colour initialisation by chromaticity clustering (Sec. 5.1) on the GPU
against the oracle, through the C ABI: the number of clusters and their centres
bit for bit (every decision is an FP64 comparison taken identically on both
sides), every pixel's id bit for bit, the mean colours within 1e-12 relative
(FP64 sums in a different order).  Then the whole "frames in" path: a clip
clustered on its first frame and decomposed with the later frames' ids taken
from the current colours on the device."""
import sys

import numpy as np
import pytest

import oracle as O
from oracle import clustering as CL
from parity import compare_frame
from scenes import make_clip, workload_clip

pytestmark = pytest.mark.gpu
P = O.default_params()


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


def _check(torch, frame, k_max=10, label=""):
    import paper_1908_01961_amd as G
    ids_g, cols_g, cen_g = G.cluster_frame(torch.from_numpy(np.ascontiguousarray(frame)).cuda(), k_max)
    ids_o, cols_o, cen_o = CL.cluster_frame(frame, k_max, P)
    ids_g = ids_g.cpu().numpy()
    _say(f"{label}: {len(cen_g)} clusters (oracle {len(cen_o)}), ids differ at {int((ids_g != ids_o).sum())}")
    assert len(cen_g) == len(cen_o)
    assert np.array_equal(cen_g, cen_o)
    assert np.array_equal(ids_g, ids_o)
    assert np.abs(cols_g - cols_o).max() <= 1e-12 * np.abs(cols_o).max()
    return ids_g, cols_g


def test_three_colour_image(torch):
    cols = np.array([[0.8, 0.2, 0.2], [0.2, 0.7, 0.3], [0.25, 0.3, 0.85]])
    lab = np.zeros((37, 45), int)
    lab[:, 15:30] = 1
    lab[:, 30:] = 2
    rng = np.random.default_rng(3)
    I = (cols[lab].transpose(2, 0, 1) * (0.3 + 0.7 * rng.random((37, 45)))[None]).astype(np.float32)
    ids, c = _check(torch, I, 10, "three colours 45x37")
    assert len(c) == 3


@pytest.mark.parametrize("name,frame_t", [("video_640x480_k6", 0), ("video_1920x1080_k10", 0)])
def test_workload_first_frames(torch, name, frame_t):
    clip = workload_clip(name, nframes=frame_t + 1, gt=False, workers=8)
    _check(torch, clip.frames[frame_t], 10, f"{name} frame {frame_t}")


@pytest.mark.parametrize("W,H,K,kmax", [(1, 1, 1, 1), (7, 3, 2, 16), (130, 67, 5, 4), (333, 200, 8, 10)])
def test_edge_shapes_and_bounds(torch, W, H, K, kmax):
    c = make_clip(W, H, K, 1, 600 + W, gt=False)
    _check(torch, c.frames[0], kmax, f"{W}x{H} K={K} k_max={kmax}")


def test_non_finite_frame_is_rejected(torch):
    import paper_1908_01961_amd as G
    c = make_clip(40, 30, 3, 1, 9, gt=False)
    f = c.frames[0].copy()
    f[1, 7, 9] = np.inf
    with pytest.raises(G.GidError) as e:
        G.cluster_frame(torch.from_numpy(f).cuda(), 10)
    assert e.value.status == 4


def test_frames_in_pipeline(torch):
    """Cluster frame 0, decompose it with the clustered ids and colours, then
    frames 1 and 2 with ids=NULL (nearest chromaticity to the current colours,
    on the device): frame 0 free-running and frames 1-2 anchored to the oracle's
    previous result, each within the schedule bar."""
    import paper_1908_01961_amd as G
    _say("frames-in pipeline 160x120 K=5 scene, 3 frames, 3x8")
    clip = make_clip(160, 120, 5, 3, 77)
    ids0, cols = _check(torch, clip.frames[0], 10, "pipeline frame 0")
    K = len(cols)
    p32 = O.default_params(state_precision="f32")
    s = G.Solver(clip.width, clip.height, G.default_params(K, gn_iters=3, pcg_iters=8, temporal=1, record_energy=1))
    s.set_base_colors(cols)
    layers = torch.empty((K + 4, clip.height, clip.width), dtype=torch.float32, device="cuda")
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    b, st = s.decompose_frame(dev(clip.frames[0]), dev(ids0), layers)
    ref0 = O.decompose_frame(clip.frames[0], ids0, cols, cols, p32, 3, 8, keep_starts=True)
    compare_frame(layers.cpu().numpy().astype(np.float64), b, st["energy_final"], ref0, 8, "pipeline frame 0:", _say)
    prev = ref0
    for t in (1, 2):
        u32 = prev.u.astype(np.float32)
        s.set_base_colors(cols)
        s.set_prev_frame(dev(clip.frames[t - 1]), dev(u32[:3]))
        s.set_state(dev(u32), prev.b)
        b, st = s.decompose_frame(dev(clip.frames[t]), None, layers)
        kw = dict(u0=u32.astype(np.float64), prev=(prev.fd.C, u32[:3].astype(np.float64)))
        ref = O.decompose_frame(clip.frames[t], None, prev.b, cols, p32, 3, 8, keep_starts=True, **kw)
        # the oracle assigned the ids from the same colours
        assert np.array_equal(ref.fd.ids, CL.nearest_ids(clip.frames[t], prev.b, P))
        compare_frame(layers.cpu().numpy().astype(np.float64), b, st["energy_final"], ref, 8,
                      f"pipeline frame {t} (ids on the device):", _say)
        prev = ref
    s.close()
