"""The base-colour step (B-step): one Gauss-Newton step on the K base colours with
the layers fixed (Sec. 6.3, eq. basecolorrefinement, and Sec. 7.1, second half).

Readings of eq. basecolorrefinement used here (the paper's printed form is
ambiguous; the reasons are given in the design notes):
  * the unknown Delta b_k is the total refinement of the initially estimated
    colour b_k^init, so the current colour is b_k = b_k^init + Delta b_k;
  * the intensity regulariser lam_IR |Delta b_k|^2 and the chromaticity
    regulariser lam_CR |C(b_k^init + Delta b_k) - C(b_k^init)|^2 both measure
    the distance from the initial estimate (cr_mode "chroma"); the printed
    chromaticity term reduces to |Delta b_k|^2 (cr_mode "literal");
  * the data sum of E_refine is taken per pixel (divided by the pixel count), so
    that the two regularisers act at the scale the paper describes them for
    (bstep_scale "pixel"); bstep_scale "sum" keeps the printed pixel sum.
The data residual I_c - R_c sum_k b_kc T_k is linear in b, so one step solves
  (A/N + lam_IR I + lam_CR sum_k J_k^T J_k) db
      = h/N - lam_IR (b - b_init) - lam_CR sum_k J_k^T (C(b_k) - C(b_k^init)),
with A, h the per-channel data blocks summed over all N pixels (the dense part
of the Jacobian, Sec. 7) and J_k = dC/dv at b_k.  b_0 = white is never refined.
The paper solves this small system by SVD on the CPU; so does the oracle
(pseudo-inverse, rcond 1e-12).  A step that would make any colour component
fall to 1e-4 or below, or that is not finite, is rejected (db = 0).

Unknown ordering: index 3 (k-1) + c for colour k = 1..K and channel c.
"""
from __future__ import annotations

import numpy as np

from .energy import chromaticity, shading
from .params import OracleParams


def bstep_sums(u: np.ndarray, b: np.ndarray, I: np.ndarray, p: OracleParams):
    """Per-channel data blocks A[c, k, l] = lam_d sum_x R_c^2 T_k T_l and
    h[c, k] = lam_d sum_x R_c T_k (I_c - R_c S_c), for k, l = 1..K."""
    u = np.asarray(u, np.float64)
    r, T = u[:3], u[3:]
    R = np.exp(r)
    e = np.asarray(I, np.float64) - R * shading(T, b)
    Tk = T[1:].reshape(T.shape[0] - 1, -1)
    K = Tk.shape[0]
    A = np.zeros((3, K, K))
    h = np.zeros((3, K))
    for c in range(3):
        Rc = R[c].ravel()
        A[c] = p.lam_data * (Tk * Rc ** 2) @ Tk.T
        h[c] = p.lam_data * Tk @ (Rc * e[c].ravel())
    return A, h


def chroma_jacobian(v: np.ndarray) -> np.ndarray:
    """dC/dv at v for C(v) = v / mean(v): (I - C 1^T / 3) / mean(v)."""
    m = v.mean()
    C = v / m
    return (np.eye(3) - np.outer(C, np.ones(3)) / 3.0) / m


def bstep_system(A: np.ndarray, h: np.ndarray, b: np.ndarray, b_init: np.ndarray, p: OracleParams,
                 npix: int):
    """The 3K x 3K normal matrix and right-hand side of the B-step."""
    K = A.shape[1]
    N = 3 * K
    H = np.zeros((N, N))
    g = np.zeros(N)
    if p.bstep_scale == "pixel":
        scale = 1.0 / npix
    elif p.bstep_scale == "sum":
        scale = 1.0
    else:
        raise ValueError(p.bstep_scale)
    for c in range(3):
        for k in range(K):
            g[3 * k + c] = h[c, k] * scale
            for l in range(K):
                H[3 * k + c, 3 * l + c] += A[c, k, l] * scale
    dtot = (np.asarray(b, np.float64) - np.asarray(b_init, np.float64)).ravel()
    H += p.lam_ir * np.eye(N)
    g -= p.lam_ir * dtot
    if p.cr_mode == "literal":
        H += p.lam_cr * np.eye(N)
        g -= p.lam_cr * dtot
    else:
        Cb = chromaticity(np.asarray(b, np.float64).T[:, :, None], p)[:, :, 0].T     # (K, 3)
        C0 = chromaticity(np.asarray(b_init, np.float64).T[:, :, None], p)[:, :, 0].T
        for k in range(K):
            Jk = chroma_jacobian(np.asarray(b[k], np.float64))
            s = slice(3 * k, 3 * k + 3)
            H[s, s] += p.lam_cr * Jk.T @ Jk
            g[s] -= p.lam_cr * Jk.T @ (Cb[k] - C0[k])
    return H, g


def bstep_solve(H: np.ndarray, g: np.ndarray, rcond: float = 1e-12) -> np.ndarray:
    """SVD pseudo-inverse solve (Sec. 7.1 solves the small system by SVD)."""
    U, s, Vt = np.linalg.svd(H)
    keep = s > rcond * s[0]
    inv = np.where(keep, 1.0 / np.where(keep, s, 1.0), 0.0)
    return Vt.T @ (inv * (U.T @ g))


def bstep(u, b, b_init, I, p: OracleParams):
    """Return (refined base colours, accepted flag)."""
    A, h = bstep_sums(u, b, I, p)
    npix = int(np.asarray(I).shape[1] * np.asarray(I).shape[2])
    H, g = bstep_system(A, h, b, b_init, p, npix)
    db = bstep_solve(H, g)
    nb = np.asarray(b, np.float64) + db.reshape(-1, 3)
    if not np.all(np.isfinite(nb)) or np.any(nb <= 1e-4):
        return np.asarray(b, np.float64).copy(), False
    return nb, True
