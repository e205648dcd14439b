"""Reflectance correction of a misclustered region by sparsity (Sec. 5.2.2), in
float64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Once a region of a frame is identified (the paper's user clicks, flood fill and
tracking, Sec. 5.2.1, are outside this restatement; the region comes in as a
mask), every base colour is tried as the region's reflectance: the region's
cluster ids are set to that colour and the frame is decomposed in full; the
illumination sparsity term of Sec. 6.2 (eq. shading-sparsity-term),
lambda_is sum_x sum_{k>=1} |T_k(x)|, is summed over the region; the colour
giving the sparsest indirect layers is kept (ties: the lowest index).

Readings: each candidate decomposition is a first-frame solve of the frame with
the fixed schedule (G outer iterations of P PCG iterations, base-colour
refinement every iteration) from the same colours, which are also the
refinement's initial estimate.
"""
from __future__ import annotations

import numpy as np

from .params import OracleParams
from .schedule import decompose_frame


def region_sparsity(u: np.ndarray, region: np.ndarray, p: OracleParams) -> float:
    """lambda_is sum over the region of sum_{k>=1} |T_k|."""
    T = np.asarray(u, np.float64)[4:]
    m = np.asarray(region, bool)
    return float(p.lam_isparsity * np.abs(T[:, m]).sum())


def correct_region(I, ids, region, b, p: OracleParams, G: int, P: int):
    """Returns (best colour index, sparsity per candidate (K,), corrected ids)."""
    ids = np.asarray(ids)
    region = np.asarray(region, bool)
    b = np.asarray(b, np.float64)
    K = b.shape[0]
    sp = np.zeros(K)
    for j in range(K):
        ids_j = np.where(region, j, ids).astype(ids.dtype)
        res = decompose_frame(I, ids_j, b, b, p, G, P, record=False)
        sp[j] = region_sparsity(res.u, region, p)
    best = int(np.argmin(sp))
    return best, sp, np.where(region, best, ids).astype(ids.dtype)
