"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics:
closed-form energy values, finite differences, an independent explicit Jacobian,
a textbook graph Laplacian, library solves (dense solve, lstsq), the IRLS bound,
exact recovery on a degenerate scene and the paper's qualitative properties.
CPU only."""
import math
import os

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import laplacian

import oracle as O
from oracle.basecolor import bstep, bstep_sums, bstep_system, bstep_solve, chroma_jacobian
from oracle.energy import (FrameData, WINDOW, energy_terms, prepare_frame, total_energy,
                           chromaticity, delta_chroma, soft_retinex_weight, intensity)
from oracle.explicit import assemble_residuals
from oracle.gauss_newton import apply_normal, jacobi_diag, linearise, pcg, rhs, surrogate_energy
from scenes import make_clip, workload_clip

P = O.default_params()
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _fd(I, ids, wsr=None, p=P):
    fd = prepare_frame(I, ids, p)
    if wsr is not None:
        fd.wsr = np.asarray(wsr, np.float64)
    return fd


def _random_problem(W=6, H=5, K=3, seed=3, temporal=True):
    c = make_clip(W, H, K, 2, seed)
    rng = np.random.default_rng(seed)
    prev = (chromaticity(c.frames[0].astype(np.float64), P), c.gt_r[0].astype(np.float64)) if temporal else (None, None)
    fd = prepare_frame(c.frames[1], c.ids[1], P, *prev)
    u = np.concatenate([c.gt_r[1], c.gt_T[1]]).astype(np.float64)
    u += 0.05 * rng.standard_normal(u.shape)
    return c, fd, u


# ---------------------------------------------------------------- parameters

def test_parameters_match_paper_fixture():
    vals = {}
    with open(os.path.join(GOLDEN, "paper_parameters.txt")) as f:
        for line in f:
            line = line.split("#")[0].split()
            if line:
                vals[line[0]] = float(line[1])
    for k, v in vals.items():
        if k == "pcg_steps_paper":
            continue
        assert getattr(P, k) == v, k


# ---------------------------------------------------------- closed-form energies

def test_data_term_vanishes_on_exact_rendering():
    rng = np.random.default_rng(0)
    K, H, W = 3, 4, 5
    b = rng.uniform(0.1, 0.9, (K, 3))
    u = np.concatenate([rng.uniform(-1, 0, (3, H, W)), rng.uniform(0, 1, (K + 1, H, W))])
    B = np.vstack([np.ones(3), b])
    I = np.exp(u[:3]) * np.einsum("kc,khw->chw", B, u[3:])
    fd = _fd(I, np.zeros((H, W), int))
    assert energy_terms(u, b, fd, P)["data"] < 1e-20


def test_hand_values_2x2_and_3x2():
    b = np.array([[0.3, 0.6, 0.9]])
    ids = np.zeros((2, 2), int)
    # 2x2, R = 1 (r = 0), T0 = 0.4, T1 = 0: data residual 0.1 per channel and pixel
    u = np.zeros((5, 2, 2))
    u[3] = 0.4
    I = np.full((3, 2, 2), 0.5)
    t = energy_terms(u, b, _fd(I, ids, wsr=np.ones((2, 2))), P)
    assert t["data"] == pytest.approx(5000 * 4 * 3 * 0.01, rel=1e-12)
    assert t["rsparsity"] == 0 and t["smooth"] == 0        # constant fields
    assert t["mono"] == pytest.approx(0.0, abs=1e-24)       # grey shading
    assert t["isparsity"] == 0 and t["nonneg"] == 0
    assert t["cluster"] == pytest.approx(200 * 4 * (np.log(b[0]) ** 2).sum(), rel=1e-12)
    # non-negativity: one layer value -0.1 costs lam_nn * 0.1; as T1 it also costs lam_is * 0.1
    u2 = u.copy()
    u2[4, 0, 0] = -0.1
    t2 = energy_terms(u2, b, _fd(I, ids, wsr=np.zeros((2, 2))), P)
    assert t2["nonneg"] == pytest.approx(1000 * 0.1, rel=1e-12)
    assert t2["isparsity"] == pytest.approx(3 * 0.1, rel=1e-12)
    # smoothness of that isolated value: |dx| at (0,0) and |dy| at (0,0): 2 * 0.1
    assert t2["smooth"] == pytest.approx(3 * 0.2, rel=1e-12)
    # monochrome: S = b_1 at one pixel: sum (S_c - 0.6)^2 = 0.18, times w_SR
    u3 = np.zeros((5, 2, 2))
    u3[4, 1, 1] = 1.0
    t3 = energy_terms(u3, b, _fd(I, ids, wsr=np.full((2, 2), 0.5)), P)
    assert t3["mono"] == pytest.approx(10 * 0.5 * 0.18, rel=1e-12)
    # 3x2 frame with a one-step edge of height h in r_0 between columns 1 and 2:
    # |grad r| = h at the two pixels left of the edge, zero elsewhere
    h = 0.7
    u4 = np.zeros((5, 2, 3))
    u4[0, :, 2] = h
    t4 = energy_terms(u4, b, _fd(np.ones((3, 2, 3)), np.zeros((2, 3), int)), P)
    assert t4["rsparsity"] == pytest.approx(20 * 2 * h, rel=1e-12)


def test_temporal_term_hand_value():
    b = np.array([[0.5, 0.5, 0.5]])
    I = np.full((3, 2, 2), 0.5)
    ids = np.zeros((2, 2), int)
    C = chromaticity(I, P)
    prev_r = np.zeros((3, 2, 2))
    fd = prepare_frame(I, ids, P, C, prev_r)
    # identical chromaticity: every in-image window pixel is a pair; a 2x2 frame has
    # 4 in-image window pixels around each pixel -> 16 pairs
    assert fd.gamma.sum() == 16
    u = np.zeros((5, 2, 2))
    u[:3] = 0.2
    t = energy_terms(u, b, fd, P)
    assert t["rconsist"] == pytest.approx(10 * 16 * 3 * 0.04, rel=1e-12)
    # a chromaticity change above the gate removes the pairs
    I2 = I.copy()
    I2[0] = 0.9
    fd2 = prepare_frame(I2, ids, P, C, prev_r)
    assert fd2.gamma.sum() == 0


def test_chromaticity_and_soft_retinex_closed_form():
    I = np.zeros((3, 2, 4))
    I[:, :, :2] = np.array([0.2, 0.4, 0.6])[:, None, None]
    I[:, :, 2:] = np.array([0.5, 0.5, 0.5])[:, None, None]
    C = chromaticity(I, P)
    assert np.allclose(C[:, 0, 0], [0.5, 1.0, 1.5])
    d = math.sqrt(0.25 + 0 + 0.25)
    dC = delta_chroma(C)
    assert dC[0, 1] == pytest.approx(d) and dC[0, 2] == pytest.approx(d)
    assert dC[0, 0] == 0 and dC[0, 3] == 0
    w = soft_retinex_weight(I, P)
    assert w[1, 1] == pytest.approx(1 - math.exp(-50 * d))
    assert w[0, 0] == 0
    black = np.zeros((3, 1, 1))
    assert np.allclose(chromaticity(black, P)[:, 0, 0], 1.0)


# --------------------------------------------------- Jacobian and operator pins

def test_fd_jacobian_matches_analytic():
    c, fd, u = _random_problem()
    lin = linearise(u, c.b_init, fd, P)
    F0, J = assemble_residuals(u, lin)
    Jd = J.toarray()
    h = 1e-6
    err = 0.0
    for j in range(u.size):
        e = np.zeros(u.size)
        e[j] = h
        Fp, _ = assemble_residuals(u + e.reshape(u.shape), lin)
        Fm, _ = assemble_residuals(u - e.reshape(u.shape), lin)
        err = max(err, np.abs((Fp - Fm) / (2 * h) - Jd[:, j]).max())
    assert err / np.abs(Jd).max() <= 1e-6


def test_matrix_free_equals_explicit():
    c, fd, u = _random_problem(7, 5, 4, seed=9)
    lin = linearise(u, c.b_init, fd, P)
    F, J = assemble_residuals(u, lin)
    rng = np.random.default_rng(1)
    for _ in range(3):
        pv = rng.standard_normal(u.shape)
        q1 = apply_normal(pv, lin).ravel()
        q2 = J.T @ (J @ pv.ravel())
        assert np.abs(q1 - q2).max() <= 1e-12 * np.abs(q2).max()
    g2 = -(J.T @ F)
    assert np.abs(rhs(lin).ravel() - g2).max() <= 1e-12 * np.abs(g2).max()
    d2 = np.asarray(J.multiply(J).sum(axis=0)).ravel()
    assert np.abs(jacobi_diag(lin).ravel() - d2).max() <= 1e-12 * d2.max()
    assert surrogate_energy(u, lin) == pytest.approx(float(F @ F), rel=1e-12)
    # symmetric and positive semi-definite
    a, b2 = rng.standard_normal(u.shape), rng.standard_normal(u.shape)
    assert np.vdot(a, apply_normal(b2, lin)) == pytest.approx(np.vdot(b2, apply_normal(a, lin)), rel=1e-12)
    assert np.vdot(a, apply_normal(a, lin)) >= 0


def test_smoothness_operator_is_weighted_graph_laplacian():
    zero = dict(lam_data=0.0, lam_cluster=0.0, lam_rsparsity=0.0, lam_rconsistency=0.0,
                lam_mono=0.0, lam_isparsity=0.0, lam_nonneg=0.0)
    p = O.default_params(**zero)
    c, fd, u = _random_problem(6, 4, 2, seed=5, temporal=False)
    lin = linearise(u, c.b_init, fd, p)
    H, W = fd.shape
    N = H * W
    for k in range(3):
        A = sp.lil_matrix((N, N))
        for y in range(H):
            for x in range(W):
                i = y * W + x
                if x + 1 < W:
                    A[i, i + 1] = A[i + 1, i] = p.lam_smooth * lin.wsx[k, y, x]
                if y + 1 < H:
                    A[i, i + W] = A[i + W, i] = p.lam_smooth * lin.wsy[k, y, x]
        L = laplacian(A.tocsr())
        v = np.random.default_rng(k).standard_normal(N)
        pv = np.zeros(u.shape)
        pv[3 + k] = v.reshape(H, W)
        q = apply_normal(pv, lin)
        assert np.allclose(q[3 + k].ravel(), L @ v, rtol=1e-12, atol=1e-9)
        assert np.abs(np.delete(q, 3 + k, axis=0)).max() == 0


@pytest.mark.parametrize("K", [2, 3, 4])
def test_pcg_to_convergence_equals_direct_solve(K):
    c, fd, u = _random_problem(8, 6, K, seed=20 + K)
    lin = linearise(u, c.b_init, fd, P)
    F, J = assemble_residuals(u, lin)
    A = (J.T @ J).toarray()
    d_direct = np.linalg.solve(A, -(J.T @ F)).reshape(u.shape)
    d_pcg, info = pcg(lin, iters=u.size * 4, tol_rz=1e-28)
    assert np.abs(d_pcg - d_direct).max() <= 1e-8 * max(1.0, np.abs(d_direct).max())


# -------------------------------------------------------------- base-colour step

@pytest.mark.parametrize("mode", ["chroma", "literal"])
def test_bstep_equals_lstsq_on_stacked_system(mode):
    p = O.default_params(cr_mode=mode)
    c, fd, u = _random_problem(6, 5, 3, seed=31, temporal=False)
    b = c.b_init + 0.02
    A, h = bstep_sums(u, b, fd.I, p)
    N = fd.shape[0] * fd.shape[1]
    Hm, g = bstep_system(A, h, b, c.b_init, p, N)
    db = bstep_solve(Hm, g)
    # stack the residual rows of the linearised refinement energy explicitly
    K = b.shape[0]
    R = np.exp(u[:3])
    B = np.vstack([np.ones(3), b])
    S = np.einsum("kc,khw->chw", B, u[3:])
    e = fd.I - R * S
    rows, tgt = [], []
    s = math.sqrt(p.lam_data / N)
    for y in range(fd.shape[0]):
        for x in range(fd.shape[1]):
            for ch in range(3):
                row = np.zeros(3 * K)
                for k in range(K):
                    row[3 * k + ch] = s * R[ch, y, x] * u[4 + k, y, x]
                rows.append(row)
                tgt.append(s * e[ch, y, x])
    dtot = (b - c.b_init).ravel()
    for j in range(3 * K):
        row = np.zeros(3 * K)
        row[j] = math.sqrt(p.lam_ir)
        rows.append(row)
        tgt.append(-math.sqrt(p.lam_ir) * dtot[j])
    for k in range(K):
        if mode == "literal":
            for ch in range(3):
                row = np.zeros(3 * K)
                row[3 * k + ch] = math.sqrt(p.lam_cr)
                rows.append(row)
                tgt.append(-math.sqrt(p.lam_cr) * dtot[3 * k + ch])
        else:
            Jk = chroma_jacobian(b[k])
            dc = b[k] / b[k].mean() - c.b_init[k] / c.b_init[k].mean()
            for ch in range(3):
                row = np.zeros(3 * K)
                row[3 * k:3 * k + 3] = math.sqrt(p.lam_cr) * Jk[ch]
                rows.append(row)
                tgt.append(-math.sqrt(p.lam_cr) * dc[ch])
    ref, *_ = np.linalg.lstsq(np.array(rows), np.array(tgt), rcond=None)
    assert np.abs(db - ref).max() <= 1e-10 * max(1.0, np.abs(ref).max())
    if mode == "literal":   # no chromaticity coupling: channels separate
        for ch in range(3):
            for k in range(K):
                for l in range(K):
                    for c2 in range(3):
                        if c2 != ch:
                            assert Hm[3 * k + ch, 3 * l + c2] == 0


def test_bstep_literal_is_exact_minimiser():
    """With the literal chromaticity term the step minimises the (quadratic)
    refinement energy exactly: it never increases it and zeroes its gradient."""
    p = O.default_params(cr_mode="literal")
    c, fd, u = _random_problem(6, 5, 3, seed=41, temporal=False)
    N = fd.shape[0] * fd.shape[1]
    b0 = c.b_init.copy()

    def e_ref(b):
        R = np.exp(u[:3])
        S = np.einsum("kc,khw->chw", np.vstack([np.ones(3), b]), u[3:])
        d = b - c.b_init
        return p.lam_data / N * ((fd.I - R * S) ** 2).sum() + (p.lam_ir + p.lam_cr) * (d ** 2).sum()

    b = b0 + 0.03
    for _ in range(3):
        nb, ok = bstep(u, b, c.b_init, fd.I, p)
        assert ok and e_ref(nb) <= e_ref(b) + 1e-12
        b = nb
    nb, _ = bstep(u, b, c.b_init, fd.I, p)
    assert np.abs(nb - b).max() < 1e-12


def test_refinement_moves_colours_towards_truth_at_true_layers():
    """Caption of fig. basecolorrefinement: refinement brings the base colours
    closer to ground truth.  With the layers held at their true values on a
    noise-free scene, B-steps reduce |b - b_true|."""
    c = make_clip(48, 32, 4, 1, 77, noise=0.0, amp=0.35)
    fd = prepare_frame(c.frames[0], c.ids[0], P)
    u = np.concatenate([c.gt_r[0], c.gt_T[0]]).astype(np.float64)
    b = c.b_init.copy()
    e0 = np.linalg.norm(b - c.b_gt)
    for _ in range(5):
        b, ok = bstep(u, b, c.b_init, fd.I, P)
        assert ok
    assert np.linalg.norm(b - c.b_gt) < e0


# ----------------------------------------------------------------- IRLS bound

def test_irls_surrogate_bound():
    c, fd, u = _random_problem(7, 6, 3, seed=51)
    u[4:] -= 0.05          # put some layers below zero so the non-negativity rows are active
    lin = linearise(u, c.b_init, fd, P)
    E = total_energy(u, c.b_init, fd, P)
    Et = surrogate_energy(u, lin)
    H, W = fd.shape
    K = u.shape[0] - 4
    n_rs = H * W - 1                                  # every pixel but the last has a forward neighbour
    n_is = K * H * W
    n_sm = (K + 1) * (H * (W - 1) + (H - 1) * W)
    n_nn = (K + 1) * H * W
    bound = P.eps_irls * (P.lam_rsparsity * n_rs + P.lam_isparsity * n_is + P.lam_smooth * n_sm) \
        + P.eps_nonneg * P.lam_nonneg * n_nn
    assert Et <= E + 1e-9
    assert E - Et <= bound


# -------------------------------------------------- exact recovery, properties

def test_single_region_exact_recovery():
    """One region of colour b, constant direct light, no indirect light and no
    noise: every term is zero at the truth, so it is the global minimiser."""
    c = make_clip(8, 6, 2, 1, 11, single_region=True)
    fd = prepare_frame(c.frames[0], c.ids[0], P)
    gt = np.concatenate([c.gt_r[0], c.gt_T[0]]).astype(np.float64)
    rng = np.random.default_rng(1)
    u = gt.copy()
    u[:4] += 0.02 * rng.standard_normal(u[:4].shape)
    u[4:] = np.abs(0.01 * rng.standard_normal(u[4:].shape))
    E0 = total_energy(u, c.b_gt, fd, P)
    for solver in ("direct", "pcg"):
        res = O.decompose_frame(c.frames[0], c.ids[0], c.b_gt, c.b_gt, P, 25, 200, u0=u,
                                refine=False, solver=solver)
        assert res.energy < 1e-8 * E0
        assert np.abs(res.u - gt).max() < 1e-4


def test_sparsity_prior_confines_indirect_layers():
    """Sec. 8.2 (evaluation of the sparsity prior) ablation: without the indirect-sparsity prior more
    pixels carry indirect light."""
    c = workload_clip("single_64x48_k4")
    def active(lam):
        p = O.default_params(lam_isparsity=lam)
        r = O.decompose_clip(c.frames, c.ids, c.b_init, p, 5, 10, temporal=False)[0]
        return (r.u[4:] > 0.01).mean()
    assert active(0.0) > active(3.0)


def test_schedule_runs_and_records_half_steps():
    c = workload_clip("single_64x48_k4")
    r = O.decompose_clip(c.frames, c.ids, c.b_init, P, 5, 10, temporal=False)[0]
    assert [e[0] for e in r.energies] == ["T", "B"] * 5
    assert np.isfinite(r.energy) and r.energy == r.energies[-1][1]
    E0 = total_energy(O.init_state(c.frames[0], c.ids[0], c.b_init), c.b_init, r.fd, P)
    assert r.energy < 0.5 * E0
    assert all(i["iters"] == 10 for i in r.pcg)


def test_generator_is_seeded_and_in_range():
    a = make_clip(40, 30, 5, 3, 123)
    b = make_clip(40, 30, 5, 3, 123)
    assert np.array_equal(a.frames, b.frames) and np.array_equal(a.ids, b.ids)
    assert a.ids.max() < 5 and a.frames.dtype == np.float32
    assert 0.3 - 1e-9 <= a.gt_T[:, 0].min() and a.gt_T[:, 0].max() <= 1.0 + 1e-6
    assert (a.b_gt >= 0.1).all() and (a.b_gt <= 0.9).all()
    assert (a.b_init >= 0.05).all() and (a.b_init <= 0.95).all()
    assert (a.gt_T[:, 1:] >= 0).all() and a.gt_T[:, 1:].max() <= 0.2
