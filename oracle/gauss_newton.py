"""The layer step (T-step): one IRLS-reweighted Gauss-Newton step on the per-pixel
unknowns with the base colours fixed, its normal equations solved by
Jacobi-preconditioned conjugate gradients (Sec. 6.4 and Sec. 7.1).

IRLS (Sec. 6.4): an l_p term |x|_p is replaced by |x|_2^2 * |x_old|_2^(p-2), with
x_old taken at the current iterate; the weights are frozen for the whole
Gauss-Newton step.  The l1 terms use (|x_old| + eps)^(-1); the non-negativity term
uses 0 if T_old > 0 else (|T_old| + eps)^(-1) (Sec. 6.4.1).

With the weights frozen the energy is a sum of squared residuals ||F(u)||^2 and
Gauss-Newton solves J^T J delta = -J^T F (Sec. 7, eq. optimization and the
normal equations after it), then sets u <- u + delta.  Here J^T J and -J^T F are
applied matrix-free, term by term; the explicit row-by-row assembly in
explicit.py is the independent check of these formulas.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .energy import (FrameData, cluster_log_reflectance, forward_diff, full_basis, intensity,
                     rgrad_norm, shading, spatial_degree, spatial_laplacian, spatial_sq)
from .params import OracleParams


@dataclass
class Linearisation:
    """Quantities frozen at u_old for one Gauss-Newton step."""

    u_old: np.ndarray
    b: np.ndarray
    fd: FrameData
    p: OracleParams
    R: np.ndarray      # (3, H, W) exp(r_old)
    S: np.ndarray      # (3, H, W) shading at u_old
    B: np.ndarray      # (K+1, 3) basis with white first
    Bc: np.ndarray     # (K+1, 3) B minus its channel mean (row 0 is zero)
    wrs: np.ndarray    # (H, W) reflectance-gradient IRLS weight
    wis: np.ndarray    # (K+1, H, W) indirect-sparsity IRLS weight (row 0 is zero)
    wnn: np.ndarray    # (K+1, H, W) non-negativity weight
    wsx: np.ndarray    # (K+1, H, W-1) smoothness weight, x direction
    wsy: np.ndarray    # (K+1, H-1, W) smoothness weight, y direction
    gsum: np.ndarray   # (H, W) number of active temporal pairs


def linearise(u_old: np.ndarray, b: np.ndarray, fd: FrameData, p: OracleParams) -> Linearisation:
    u_old = np.asarray(u_old, np.float64)
    r, T = u_old[:3], u_old[3:]
    B = full_basis(b)
    Bc = B - B.mean(axis=1, keepdims=True)
    wrs = (rgrad_norm(r) + p.eps_irls) ** (p.p - 2.0)
    wis = 1.0 / (np.abs(T) + p.eps_irls)
    wis[0] = 0.0                                   # the direct layer has no sparsity prior
    wnn = np.where(T > 0.0, 0.0, 1.0 / (np.abs(T) + p.eps_nonneg))
    gx, gy = forward_diff(T)
    wsx = 1.0 / (np.abs(gx) + p.eps_irls)
    wsy = 1.0 / (np.abs(gy) + p.eps_irls)
    gsum = fd.gamma.sum(axis=0) if fd.gamma is not None else np.zeros(T.shape[1:])
    return Linearisation(u_old, np.asarray(b, np.float64), fd, p, np.exp(r), shading(T, b), B, Bc,
                         wrs, wis, wnn, wsx, wsy, gsum)


def _stencil_apply(f: np.ndarray, wx: np.ndarray, wy: np.ndarray) -> np.ndarray:
    """sum over forward pairs (x, x+e_d) of w(x) (f(x+e_d) - f(x)) (e_{x+e_d} - e_x):
    the normal-equation block of a weighted squared forward difference."""
    q = np.zeros_like(f)
    ex = wx * (f[..., :, 1:] - f[..., :, :-1])
    q[..., :, 1:] += ex
    q[..., :, :-1] -= ex
    ey = wy * (f[..., 1:, :] - f[..., :-1, :])
    q[..., 1:, :] += ey
    q[..., :-1, :] -= ey
    return q


def apply_normal(pv: np.ndarray, lin: Linearisation) -> np.ndarray:
    """q = J^T J p for the frozen-weight residuals at u_old."""
    P = lin.p
    pr, pT = pv[:3], pv[3:]
    R, S, B, Bc = lin.R, lin.S, lin.B, lin.Bc
    q = np.zeros_like(pv)
    qr, qT = q[:3], q[3:]
    # data: row_c = -sqrt(l) R_c (S_c dr_c + sum_k b_kc dT_k)
    a = R * (S * pr + np.einsum("kc,khw->chw", B, pT))
    qr += P.lam_data * R * S * a
    qT += P.lam_data * np.einsum("kc,chw->khw", B, R * a)
    # clustering and temporal consistency: unary on r
    qr += P.lam_cluster * pr
    qr += P.lam_rconsistency * lin.gsum[None] * pr
    # spatial consistency pairs: a constant-weight graph Laplacian on r
    if lin.fd.sp_edges is not None:
        qr += P.lam_rconsistency * spatial_laplacian(pr, lin.fd.sp_edges)
    # monochrome: row_c = sqrt(l w_SR) sum_k (b_kc - mean_c b_k) dT_k
    m = np.einsum("kc,khw->chw", Bc, pT)
    qT += P.lam_mono * lin.fd.wsr[None] * np.einsum("kc,chw->khw", Bc, m)
    # indirect sparsity and non-negativity: unary on T_k
    qT += (P.lam_isparsity * lin.wis + P.lam_nonneg * lin.wnn) * pT
    # reflectance sparsity: one weight per pixel shared by channels and directions
    wrs = P.lam_rsparsity * lin.wrs
    qr += _stencil_apply(pr, wrs[None, :, :-1], wrs[None, :-1, :])
    # smoothness: one weight per layer, pixel and direction
    qT += _stencil_apply(pT, P.lam_smooth * lin.wsx, P.lam_smooth * lin.wsy)
    return q


def rhs(lin: Linearisation) -> np.ndarray:
    """g = -J^T F at u_old."""
    P, fd = lin.p, lin.fd
    u = lin.u_old
    r, T = u[:3], u[3:]
    R, S, B, Bc = lin.R, lin.S, lin.B, lin.Bc
    g = np.zeros_like(u)
    gr, gT = g[:3], g[3:]
    e = fd.I - R * S
    gr += P.lam_data * R * S * e
    gT += P.lam_data * np.einsum("kc,chw->khw", B, R * e)
    gr -= P.lam_cluster * (r - cluster_log_reflectance(lin.b, fd.ids))
    if fd.gamma is not None:
        for o in range(9):
            gr -= P.lam_rconsistency * fd.gamma[o][None] * (r - fd.rprev[o])
    if fd.sp_edges is not None:
        gr -= P.lam_rconsistency * spatial_laplacian(r, fd.sp_edges)
    mdev = S - intensity(S)[None]
    gT -= P.lam_mono * fd.wsr[None] * np.einsum("kc,chw->khw", Bc, mdev)
    gT -= (P.lam_isparsity * lin.wis + P.lam_nonneg * lin.wnn) * T
    wrs = P.lam_rsparsity * lin.wrs
    gr -= _stencil_apply(r, wrs[None, :, :-1], wrs[None, :-1, :])
    gT -= _stencil_apply(T, P.lam_smooth * lin.wsx, P.lam_smooth * lin.wsy)
    return g


def jacobi_diag(lin: Linearisation) -> np.ndarray:
    """diag(J^T J): the squared column norms of J, term by term."""
    P = lin.p
    R, S, B, Bc = lin.R, lin.S, lin.B, lin.Bc
    n = lin.u_old.shape[0]
    d = np.zeros((n,) + R.shape[1:])
    dr, dT = d[:3], d[3:]
    dr += P.lam_data * (R * S) ** 2
    dT += P.lam_data * np.einsum("kc,chw->khw", B ** 2, R ** 2)
    dr += P.lam_cluster + P.lam_rconsistency * lin.gsum[None]
    if lin.fd.sp_edges is not None:
        dr += P.lam_rconsistency * spatial_degree(lin.fd.sp_edges)[None]
    dT += P.lam_mono * lin.fd.wsr[None] * (Bc ** 2).sum(axis=1)[:, None, None]
    dT += P.lam_isparsity * lin.wis + P.lam_nonneg * lin.wnn

    def pair_sum(wx, wy):
        s = np.zeros(wx.shape[:-2] + R.shape[1:])
        s[..., :, :-1] += wx
        s[..., :, 1:] += wx
        s[..., :-1, :] += wy
        s[..., 1:, :] += wy
        return s

    wrs = P.lam_rsparsity * lin.wrs
    dr += pair_sum(wrs[:, :-1], wrs[:-1, :])[None]
    dT += pair_sum(P.lam_smooth * lin.wsx, P.lam_smooth * lin.wsy)
    return d


def surrogate_energy(u: np.ndarray, lin: Linearisation) -> float:
    """||F(u)||^2 with the weights frozen at lin.u_old (the IRLS surrogate)."""
    P, fd = lin.p, lin.fd
    u = np.asarray(u, np.float64)
    r, T = u[:3], u[3:]
    R = np.exp(r)
    S = shading(T, lin.b)
    e = P.lam_data * ((fd.I - R * S) ** 2).sum()
    e += P.lam_cluster * ((r - cluster_log_reflectance(lin.b, fd.ids)) ** 2).sum()
    gx, gy = forward_diff(r)
    e += P.lam_rsparsity * ((lin.wrs[None, :, :-1] * gx ** 2).sum() + (lin.wrs[None, :-1, :] * gy ** 2).sum())
    if fd.gamma is not None:
        for o in range(9):
            e += P.lam_rconsistency * (fd.gamma[o][None] * (r - fd.rprev[o]) ** 2).sum()
    if fd.sp_edges is not None:
        e += P.lam_rconsistency * spatial_sq(r, fd.sp_edges)
    e += P.lam_mono * (fd.wsr * ((S - intensity(S)[None]) ** 2).sum(axis=0)).sum()
    e += ((P.lam_isparsity * lin.wis + P.lam_nonneg * lin.wnn) * T ** 2).sum()
    tx, ty = forward_diff(T)
    e += P.lam_smooth * ((lin.wsx * tx ** 2).sum() + (lin.wsy * ty ** 2).sum())
    return float(e)


def pcg(lin: Linearisation, iters: int, *, tol_rz: float = 0.0, g: np.ndarray | None = None,
        diag: np.ndarray | None = None):
    """Jacobi-preconditioned CG on J^T J delta = g from delta = 0, for a fixed
    number of iterations (Sec. 7.1 uses a fixed count of data-parallel PCG steps;
    the preconditioner and stopping rule are the readings noted in the design).

    Breakdown guards: stop before the update if <p, q> is not positive and
    finite; stop after it if <r, z> becomes zero (or falls below tol_rz).
    Returns (delta, info) with the final <r, z> and the iteration count.
    """
    g = rhs(lin) if g is None else g
    M = jacobi_diag(lin) if diag is None else diag
    delta = np.zeros_like(g)
    r = g.copy()
    z = r / M
    pv = z.copy()
    rz = float(np.vdot(r, z))
    done = 0
    for _ in range(iters):
        q = apply_normal(pv, lin)
        pq = float(np.vdot(pv, q))
        if not (pq > 0.0) or not np.isfinite(pq):
            break
        alpha = rz / pq
        delta += alpha * pv
        r -= alpha * q
        z = r / M
        rz_new = float(np.vdot(r, z))
        done += 1
        if rz_new == 0.0 or rz_new <= tol_rz:
            rz = rz_new
            break
        beta = rz_new / rz
        pv = z + beta * pv
        rz = rz_new
    return delta, dict(rz=rz, iters=done)
