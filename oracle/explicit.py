"""Row-by-row residual vector F and sparse Jacobian J of the frozen-weight
(IRLS) least-squares problem of one layer step, and the direct Gauss-Newton
solve J^T J delta = -J^T F (Sec. 7, the normal equations after eq. optimization).

This is an independent second statement of the residuals listed with the energy
of Sec. 6 (one Python loop per pixel, one row per residual), used to check the
matrix-free formulas in gauss_newton.py and as the exact linear solver on small
frames.  Column j of J is unknown j // Npx at pixel j % Npx (planar order).
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .energy import SPATIAL_DIRS, full_basis
from .gauss_newton import Linearisation


def assemble_residuals(u: np.ndarray, lin: Linearisation):
    """F(u) and J(u) = dF/du with the weights frozen at lin.u_old.

    The set of rows depends only on the frame shape, the temporal gates and
    K, never on u, so F at two different u can be compared row by row.
    """
    P, fd = lin.p, lin.fd
    u = np.asarray(u, np.float64)
    n, H, W = u.shape
    K = n - 4
    N = H * W
    B = full_basis(lin.b)
    mu = B.mean(axis=1)
    lnb = np.log(lin.b)
    F, ri, ci, vals = [], [], [], []

    def col(comp, y, x):
        return comp * N + y * W + x

    def add_row(fval, entries):
        i = len(F)
        F.append(fval)
        for c_, v_ in entries:
            ri.append(i)
            ci.append(c_)
            vals.append(v_)

    sd = math.sqrt(P.lam_data)
    scl = math.sqrt(P.lam_cluster)
    src = math.sqrt(P.lam_rconsistency)
    for y in range(H):
        for x in range(W):
            r = u[0:3, y, x]
            T = u[3:, y, x]
            R = np.exp(r)
            S = [sum(B[k, c] * T[k] for k in range(K + 1)) for c in range(3)]
            for c in range(3):                                   # data fidelity
                ent = [(col(c, y, x), -sd * R[c] * S[c])]
                ent += [(col(3 + k, y, x), -sd * R[c] * B[k, c]) for k in range(K + 1)]
                add_row(sd * (fd.I[c, y, x] - R[c] * S[c]), ent)
            idc = fd.ids[y, x]
            for c in range(3):                                   # reflectance clustering
                add_row(scl * (r[c] - lnb[idc, c]), [(col(c, y, x), scl)])
            srs = math.sqrt(P.lam_rsparsity * lin.wrs[y, x])     # reflectance sparsity
            for (dy, dx) in ((0, 1), (1, 0)):
                yy, xx = y + dy, x + dx
                if yy >= H or xx >= W:
                    continue
                for c in range(3):
                    add_row(srs * (u[c, yy, xx] - r[c]), [(col(c, yy, xx), srs), (col(c, y, x), -srs)])
            if fd.gamma is not None:                             # temporal consistency
                for o in range(9):
                    if fd.gamma[o, y, x] == 0.0:
                        continue
                    for c in range(3):
                        add_row(src * (r[c] - fd.rprev[o, c, y, x]), [(col(c, y, x), src)])
            if fd.sp_edges is not None:                          # spatial consistency pairs
                for d, (dy, dx) in enumerate(SPATIAL_DIRS):
                    yy, xx = y + dy, x + dx
                    if fd.sp_edges[d, y, x] == 0.0 or not (0 <= yy < H and 0 <= xx < W):
                        continue
                    for c in range(3):
                        add_row(src * (r[c] - u[c, yy, xx]), [(col(c, y, x), src), (col(c, yy, xx), -src)])
            smo = math.sqrt(P.lam_mono * fd.wsr[y, x])           # monochromaticity
            mS = sum(S) / 3.0
            for c in range(3):
                ent = [(col(3 + k, y, x), smo * (B[k, c] - mu[k])) for k in range(1, K + 1)]
                add_row(smo * (S[c] - mS), ent)
            for k in range(1, K + 1):                            # indirect sparsity
                s = math.sqrt(P.lam_isparsity * lin.wis[k, y, x])
                add_row(s * T[k], [(col(3 + k, y, x), s)])
            for k in range(K + 1):                               # smoothness
                if x + 1 < W:
                    s = math.sqrt(P.lam_smooth * lin.wsx[k, y, x])
                    add_row(s * (u[3 + k, y, x + 1] - T[k]), [(col(3 + k, y, x + 1), s), (col(3 + k, y, x), -s)])
                if y + 1 < H:
                    s = math.sqrt(P.lam_smooth * lin.wsy[k, y, x])
                    add_row(s * (u[3 + k, y + 1, x] - T[k]), [(col(3 + k, y + 1, x), s), (col(3 + k, y, x), -s)])
            for k in range(K + 1):                               # non-negativity
                s = math.sqrt(P.lam_nonneg * lin.wnn[k, y, x])
                add_row(s * T[k], [(col(3 + k, y, x), s)])
    J = sp.csr_matrix((vals, (ri, ci)), shape=(len(F), n * N))
    return np.asarray(F), J


def direct_step(lin: Linearisation, dense_limit: int = 4000) -> np.ndarray:
    """Exact Gauss-Newton update: solve J^T J delta = -J^T F at u_old."""
    F, J = assemble_residuals(lin.u_old, lin)
    A = (J.T @ J).tocsc()
    g = -(J.T @ F)
    if A.shape[0] <= dense_limit:
        d = np.linalg.solve(A.toarray(), g)
    else:
        d = spla.spsolve(A, g)
    return d.reshape(lin.u_old.shape)
