"""Pins of the oracle's chromaticity clustering (Sec. 5.1) against library
routines (numpy.histogramdd, scikit-learn's weighted k-means), exact recovery
of a few-colour image, and hand cases of the merge rule.  CPU only."""
import numpy as np
import pytest

import oracle as O
from oracle import clustering as CL
from oracle.energy import chromaticity

P = O.default_params()


def _regions(H=24, W=30, shading=False, seed=0):
    """Three vertical bands of distinct colours (chromaticities far apart)."""
    cols = np.array([[0.8, 0.2, 0.2], [0.2, 0.7, 0.3], [0.25, 0.3, 0.85]])
    lab = np.zeros((H, W), int)
    lab[:, W // 3:2 * W // 3] = 1
    lab[:, 2 * W // 3:] = 2
    I = cols[lab].transpose(2, 0, 1).copy()
    if shading:
        rng = np.random.default_rng(seed)
        s = 0.3 + 0.7 * rng.random((H, W))
        I = I * s[None]
    return I, lab, cols


def test_histogram_equals_histogramdd():
    rng = np.random.default_rng(1)
    I = rng.uniform(0.01, 1.0, size=(3, 40, 50))
    h = CL.chroma_histogram(I, P)
    C = chromaticity(I, P).reshape(3, -1).T
    edges = [np.linspace(0.0, 3.0, 11)] * 3
    ref, _ = np.histogramdd(C, bins=edges)
    assert h.sum() == 2000
    assert np.array_equal(h.reshape(10, 10, 10), ref.astype(np.int64))


def test_weighted_kmeans_equals_sklearn():
    from sklearn.cluster import KMeans
    rng = np.random.default_rng(2)
    # chromaticities scattered around four colours
    base = np.array([[0.9, 0.2, 0.2], [0.2, 0.8, 0.2], [0.2, 0.2, 0.9], [0.6, 0.6, 0.2]])
    lab = rng.integers(0, 4, size=(60, 70))
    I = base[lab].transpose(2, 0, 1) * (1.0 + 0.25 * rng.standard_normal((3, 60, 70)))
    I = np.abs(I) + 0.01
    hist = CL.chroma_histogram(I, P)
    K = 6
    seeds = CL.kmeans_seeds(hist, K)
    centres, assign = CL.weighted_kmeans(hist, K)
    nz = np.flatnonzero(hist)
    X = np.array([CL.bin_midpoint(b) for b in nz])
    km = KMeans(n_clusters=len(seeds), init=np.array([CL.bin_midpoint(s) for s in seeds]), n_init=1,
                algorithm="lloyd", tol=0.0, max_iter=300).fit(X, sample_weight=hist[nz].astype(np.float64))
    assert np.abs(km.cluster_centers_ - centres).max() <= 1e-10
    assert all(assign[b] == l for b, l in zip(nz, km.labels_))


def test_seeds_are_farthest_points():
    hist = np.zeros(1000, np.int64)
    a = (3 * 10 + 3) * 10 + 3          # around white
    b = (6 * 10 + 1) * 10 + 1          # red corner
    c = (4 * 10 + 3) * 10 + 3          # next to a
    hist[a], hist[b], hist[c] = 50, 5, 20
    assert CL.kmeans_seeds(hist, 2) == [a, b]
    assert CL.kmeans_seeds(hist, 3) == [a, b, c]
    assert CL.kmeans_seeds(hist, 5) == [a, b, c]   # only three non-empty bins


@pytest.mark.parametrize("shading", [False, True])
def test_three_colour_image_is_recovered(shading):
    I, lab, cols = _regions(shading=shading)
    ids, colours, centres = CL.cluster_frame(I, 10, P)
    assert len(colours) == 3
    # the same partition of the pixels
    perm = {int(ids[lab == j][0]): j for j in range(3)}
    assert len(perm) == 3
    assert np.array_equal(np.vectorize(perm.get)(ids), lab)
    for k, j in perm.items():
        assert np.allclose(centres[k], cols[j] / cols[j].mean(), atol=0.15)   # within the bin of the truth
        expect = I[:, lab == j].mean(axis=1)
        assert np.allclose(colours[k], expect, rtol=1e-12)
        if not shading:
            assert np.allclose(colours[k], cols[j], rtol=1e-12)


def test_merge_rule_hand_cases():
    hist = np.zeros(1000, np.int64)
    b1, b2, b3 = 333, 334, 600
    hist[b1], hist[b2], hist[b3] = 30, 10, 7
    m1, m2 = CL.bin_midpoint(b1), CL.bin_midpoint(b2)
    # two centres 0.15 apart: the smaller cluster (10 pixels) joins the larger;
    # the merged centre is the population-weighted mean of the two bins
    c = np.array([m1, m1 + np.array([0.0, 0.0, 0.15]), CL.bin_midpoint(b3)])
    out_c, out_a = CL.merge_clusters(c, {b1: 0, b2: 1, b3: 2}, hist, 0.2)
    assert len(out_c) == 2
    assert out_a == {b1: 0, b2: 0, b3: 1}
    assert np.allclose(out_c[0], (30 * m1 + 10 * m2) / 40, rtol=0, atol=1e-15)
    # 0.25 apart: kept
    c2 = c.copy()
    c2[1] = m1 + np.array([0.0, 0.0, 0.25])
    out_c, out_a = CL.merge_clusters(c2, {b1: 0, b2: 1, b3: 2}, hist, 0.2)
    assert len(out_c) == 3 and out_a == {b1: 0, b2: 1, b3: 2}
    # the larger cluster absorbs the smaller whatever their order
    hist2 = hist.copy()
    hist2[b1], hist2[b2] = 10, 30
    out_c, out_a = CL.merge_clusters(c, {b1: 0, b2: 1, b3: 2}, hist2, 0.2)
    assert out_a == {b1: 0, b2: 0, b3: 1}
    assert np.allclose(out_c[0], (10 * m1 + 30 * m2) / 40, rtol=0, atol=1e-15)


def test_nearest_ids_on_an_image_of_the_base_colours():
    b = np.array([[0.8, 0.2, 0.2], [0.2, 0.7, 0.3], [0.25, 0.3, 0.85]])
    lab = np.array([[0, 1, 2, 1], [2, 2, 0, 1]])
    I = (b[lab] * 0.5).transpose(2, 0, 1)         # any intensity: chromaticity decides
    assert np.array_equal(CL.nearest_ids(I, b, P), lab)


def test_clustering_a_synthetic_first_frame_finds_its_distinct_colours():
    """On a noise-free, point-sampled scene without indirect light whose colours
    are far apart in chromaticity, the clusters are the scene's colours: every
    pixel of a colour's Voronoi regions carries that colour's cluster.  (With
    box-supersampled edges the mixed edge colours populate bins of their own,
    which the upper bound K then spends clusters on.)"""
    from scenes import make_clip
    c = make_clip(96, 64, 3, 1, 7, amp=0.0, noise=0.0, supersample=False)
    Cb = c.b_gt / c.b_gt.mean(axis=1, keepdims=True)
    d = min(np.linalg.norm(Cb[i] - Cb[j]) for i in range(3) for j in range(i + 1, 3))
    if d < 0.5:
        pytest.skip("scene colours too close in chromaticity for this check")
    ids, colours, _ = CL.cluster_frame(c.frames[0], 10, P)
    assert len(colours) == 3
    for k in range(3):
        region = c.ids[0] == k
        vals = np.unique(ids[region])
        assert len(vals) == 1
