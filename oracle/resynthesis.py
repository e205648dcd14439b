"""Re-synthesis of a frame from its decomposition (Sec. 8.4), in float64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The layers recombine by the image-formation model of Sec. 4,
I = R * sum_{k=0..K} b_k T_k with b_0 white.  The live applications edit
the recombination: recolouring an object changes its base colour, which
recolours its indirect layer consistently, and its reflectance (Sec. 8.4.1);
colour keying changes the base colour of the background's indirect layer
(Sec. 8.4.2); spill suppression drops a colour's indirect layer (Sec. 8.4.3).
One rule covers all three:

    I'_c(x) = R_c(x) s_{id(x), c} (T_0(x) + sum_{k=1..K} g_k b'_{k,c} T_k(x))

with new base colours b', a gain g_k per indirect layer (0 removes it) and a
per-cluster reflectance scale s (1 leaves the reflectance alone).
"""
from __future__ import annotations

import numpy as np


def resynthesize(layers: np.ndarray, b_new: np.ndarray, gain=None, ids=None, refl_scale=None) -> np.ndarray:
    """layers: (K+4, H, W) with linear reflectance R first, then T_0..T_K;
    b_new (K, 3); gain (K,) or None; ids (H, W) and refl_scale (K, 3) or None."""
    L = np.asarray(layers, np.float64)
    K = L.shape[0] - 4
    R, T = L[:3], L[3:]
    b = np.asarray(b_new, np.float64).reshape(K, 3)
    g = np.ones(K) if gain is None else np.asarray(gain, np.float64)
    S = np.repeat(T[0][None], 3, axis=0)
    for k in range(K):
        S = S + (g[k] * b[k])[:, None, None] * T[k + 1][None]
    Rp = R.copy()
    if ids is not None and refl_scale is not None:
        s = np.asarray(refl_scale, np.float64).reshape(K, 3)
        Rp = R * s[np.asarray(ids, np.int64)].transpose(2, 0, 1)
    return Rp * S
