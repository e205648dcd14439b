"""Pins of the oracle's spatial consistency pairs (Sec. 6.1, reading): the
SplitMix64 sampler against its published output sequence, the sampled pair
set by brute force on tiny frames, the pair operator against a textbook graph
Laplacian, the chromaticity gate, and the Jacobian of the whole step with the
pairs on (central differences; matrix-free against the explicit rows).  CPU only."""
import math

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import laplacian

import oracle as O
from oracle.energy import (SPATIAL_DIRS, chromaticity, energy_terms, prepare_frame, spatial_degree,
                           spatial_edges, spatial_laplacian, spatial_sampled, splitmix64)
from oracle.explicit import assemble_residuals
from oracle.gauss_newton import apply_normal, jacobi_diag, linearise, rhs
from scenes import make_clip

PS = O.default_params(spatial_pairs=True)
GAMMA = 0x9E3779B97F4A7C15


def test_splitmix64_published_sequence():
    """SplitMix64 from state 0: the first outputs of the reference generator."""
    assert splitmix64(0) == 0xE220A8397B1DCDAF
    assert splitmix64(GAMMA) == 0x6E789E6AA1B965F4
    assert splitmix64((2 * GAMMA) & ((1 << 64) - 1)) == 0x06C45D188009454F
    xs = np.array([0, GAMMA, (2 * GAMMA) & ((1 << 64) - 1), 12345, (1 << 64) - 1], dtype=np.uint64)
    assert [int(v) for v in splitmix64(xs)] == [splitmix64(int(v)) for v in xs]


def test_sampler_keeps_about_half_of_the_edges():
    s = spatial_sampled(2019, 100, 100)
    frac = s.mean()
    assert abs(frac - 0.5) < 0.01          # 40000 Bernoulli(1/2) draws: sd 0.0025


def _brute_pairs(C, seed, gate):
    """Active pairs of a tiny frame by the definition, one edge at a time."""
    _, H, W = C.shape
    pairs = []
    for y in range(H):
        for x in range(W):
            i = y * W + x
            for d, (dy, dx) in enumerate(SPATIAL_DIRS):
                yy, xx = y + dy, x + dx
                if not (0 <= yy < H and 0 <= xx < W):
                    continue
                if splitmix64(((seed & 0xFFFFFFFF) << 32) | (4 * i + d)) >> 63:
                    continue
                if math.dist(C[:, y, x], C[:, yy, xx]) < gate:
                    pairs.append(((y, x), (yy, xx)))
    return pairs


def test_energy_term_by_brute_force_on_a_3x4_frame():
    rng = np.random.default_rng(4)
    I = np.full((3, 3, 4), 0.5)
    I[:, :, 3] = [[0.9], [0.3], [0.3]]          # a chromaticity jump: no pairs across it
    fd = prepare_frame(I, np.zeros((3, 4), int), PS)
    pairs = _brute_pairs(chromaticity(I, PS), PS.spatial_seed, PS.chroma_gate)
    assert len(pairs) > 3
    assert all((a[1] == 3) == (b[1] == 3) for a, b in pairs)
    u = np.zeros((5, 3, 4))
    u[:3] = rng.normal(0.0, 0.3, size=(3, 3, 4))
    expect = 10.0 * sum(((u[:3, a[0], a[1]] - u[:3, b[0], b[1]]) ** 2).sum() for a, b in pairs)
    t = energy_terms(u, np.array([[0.5, 0.5, 0.5]]), fd, PS)
    assert t["rconsist"] == pytest.approx(expect, rel=1e-12)
    # the pairs are off unless asked for
    fd0 = prepare_frame(I, np.zeros((3, 4), int), O.default_params())
    assert energy_terms(u, np.array([[0.5, 0.5, 0.5]]), fd0, O.default_params())["rconsist"] == 0.0


def test_pair_operator_is_a_graph_laplacian():
    c = make_clip(9, 7, 2, 1, 5)
    C = chromaticity(c.frames[0].astype(np.float64), PS)
    E = spatial_edges(C, PS)
    H, W = 7, 9
    A = np.zeros((H * W, H * W))
    for (y, x), (yy, xx) in _brute_pairs(C, PS.spatial_seed, PS.chroma_gate):
        A[y * W + x, yy * W + xx] = A[yy * W + xx, y * W + x] = 1.0
    L = laplacian(sp.csr_matrix(A)).toarray()
    f = np.random.default_rng(1).normal(size=(3, H, W))
    q = spatial_laplacian(f, E)
    for ch in range(3):
        assert np.allclose(q[ch].ravel(), L @ f[ch].ravel(), rtol=0, atol=1e-12)
    assert np.array_equal(spatial_degree(E).ravel(), A.sum(axis=1))


def _problem(seed=3):
    c = make_clip(6, 5, 3, 2, seed)
    rng = np.random.default_rng(seed)
    prev = (chromaticity(c.frames[0].astype(np.float64), PS), c.gt_r[0].astype(np.float64))
    fd = prepare_frame(c.frames[1], c.ids[1], PS, *prev)
    u = np.concatenate([c.gt_r[1], c.gt_T[1]]).astype(np.float64)
    u += 0.05 * rng.standard_normal(u.shape)
    return c, fd, u


def test_matrix_free_equals_explicit_with_spatial_pairs():
    c, fd, u = _problem()
    assert fd.sp_edges.sum() > 0
    lin = linearise(u, c.b_init, fd, PS)
    F, J = assemble_residuals(u, lin)
    A = (J.T @ J).tocsr()
    p = np.random.default_rng(2).normal(size=u.shape)
    assert np.allclose(apply_normal(p, lin).ravel(), A @ p.ravel(), rtol=1e-12, atol=1e-9)
    assert np.allclose(rhs(lin).ravel(), -(J.T @ F), rtol=1e-12, atol=1e-9)
    assert np.allclose(jacobi_diag(lin).ravel(), A.diagonal(), rtol=1e-12, atol=1e-9)


def test_fd_jacobian_with_spatial_pairs():
    c, fd, u = _problem(7)
    lin = linearise(u, c.b_init, fd, PS)
    _, J = assemble_residuals(u, lin)
    J = J.toarray()
    h = 1e-6
    rng = np.random.default_rng(0)
    for j in rng.choice(u.size, 25, replace=False):
        e = np.zeros(u.size)
        e[j] = h
        Fp, _ = assemble_residuals(u + e.reshape(u.shape), lin)
        Fm, _ = assemble_residuals(u - e.reshape(u.shape), lin)
        num = (Fp - Fm) / (2 * h)
        assert np.abs(num - J[:, j]).max() <= 1e-6 * max(1.0, np.abs(J[:, j]).max())
