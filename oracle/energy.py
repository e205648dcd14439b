"""Image-derived quantities and the true decomposition energy, in float64.

Layout: a frame is a (3, H, W) array (planar RGB); the unknowns of one frame are a
(K+4, H, W) array u = (r_0, r_1, r_2, T_0, T_1 .. T_K) where r = ln R (Sec. 6.1,
eq. clustering-term: the reflectance is optimised in the log domain) and T_0 is
the direct and T_k the indirect illumination layers (Sec. 4, eq. imageformation).
Base colours b are a (K, 3) array for k = 1..K; b_0 = (1, 1, 1) is prepended
where the image-formation sum needs it.  Cluster ids are 0-based: id = j means
base colour b_{j+1}.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Optional

import numpy as np

from .params import OracleParams

#: Offsets (dy, dx) of the 3x3 temporal window (reading of the spatio-temporal
#: consistency prior of Sec. 6.1, whose sampling the paper defers to prior work).
WINDOW = tuple((dy, dx) for dy in (-1, 0, 1) for dx in (-1, 0, 1))

#: Spatial pairs of the same prior (reading): the edges between a pixel and its
#: eight neighbours, each enumerated once from the pixel that owns it in one of
#: four forward directions d = 0..3 (right, down-right, down, down-left).  An
#: edge is sampled when the top bit of SplitMix64 of the key
#: (seed << 32) | (4 i + d), i the owning pixel's row-major index, is zero
#: (probability 1/2, the same edges at both ends and in every frame), and it is
#: active when the two pixels' chromaticities are closer than the gate.  Each
#: active edge adds lambda_rc sum_c (r_c(x) - r_c(y))^2.
SPATIAL_DIRS = ((0, 1), (1, 1), (1, 0), (1, -1))

_M64 = (1 << 64) - 1


def splitmix64(x):
    """The SplitMix64 output for state x (Steele, Lea and Flood, 2014): the
    golden-ratio increment, then the two xor-shift-multiply rounds.  Works on
    Python ints and on numpy uint64 arrays."""
    if isinstance(x, np.ndarray):
        z = x.astype(np.uint64) + np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))
    z = (x + 0x9E3779B97F4A7C15) & _M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
    return z ^ (z >> 31)


def spatial_sampled(seed: int, H: int, W: int) -> np.ndarray:
    """(4, H, W) 0/1: edge (pixel, direction d) drawn by the sampler."""
    i = np.arange(H * W, dtype=np.uint64).reshape(H, W)
    out = np.zeros((4, H, W))
    for d in range(4):
        key = (np.uint64(seed & 0xFFFFFFFF) << np.uint64(32)) | (np.uint64(4) * i + np.uint64(d))
        out[d] = (splitmix64(key) >> np.uint64(63)) == 0
    return out


def _edge_slices(H, W, dy, dx):
    """(source rows, source cols, target rows, target cols) of the in-image edges
    from (y, x) to (y + dy, x + dx)."""
    ys = slice(0, H - dy)
    xs = slice(max(0, -dx), min(W, W - dx))
    yt = slice(dy, H)
    xt = slice(max(0, -dx) + dx, min(W, W - dx) + dx)
    return ys, xs, yt, xt


def spatial_edges(C: np.ndarray, p: OracleParams) -> np.ndarray:
    """(4, H, W) 0/1 active spatial pairs owned by each pixel (see SPATIAL_DIRS)."""
    _, H, W = C.shape
    samp = spatial_sampled(p.spatial_seed, H, W)
    E = np.zeros((4, H, W))
    for d, (dy, dx) in enumerate(SPATIAL_DIRS):
        ys, xs, yt, xt = _edge_slices(H, W, dy, dx)
        diff = C[:, ys, xs] - C[:, yt, xt]
        dist = np.sqrt((diff[0] * diff[0] + diff[1] * diff[1]) + diff[2] * diff[2])
        E[d, ys, xs] = samp[d, ys, xs] * (dist < p.chroma_gate)
    return E


def spatial_laplacian(f: np.ndarray, E: np.ndarray) -> np.ndarray:
    """sum over active edges (x, y) of (f(x) - f(y)) (e_x - e_y), per channel of f (3, H, W)."""
    q = np.zeros_like(f)
    _, H, W = f.shape
    for d, (dy, dx) in enumerate(SPATIAL_DIRS):
        ys, xs, yt, xt = _edge_slices(H, W, dy, dx)
        e = E[d, ys, xs][None] * (f[:, ys, xs] - f[:, yt, xt])
        q[:, ys, xs] += e
        q[:, yt, xt] -= e
    return q


def spatial_degree(E: np.ndarray) -> np.ndarray:
    """Number of active spatial pairs at each pixel."""
    _, H, W = E.shape
    deg = np.zeros((H, W))
    for d, (dy, dx) in enumerate(SPATIAL_DIRS):
        ys, xs, yt, xt = _edge_slices(H, W, dy, dx)
        deg[ys, xs] += E[d, ys, xs]
        deg[yt, xt] += E[d, ys, xs]
    return deg


def spatial_sq(r: np.ndarray, E: np.ndarray) -> float:
    """sum over active edges of sum_c (r_c(x) - r_c(y))^2."""
    _, H, W = r.shape
    acc = 0.0
    for d, (dy, dx) in enumerate(SPATIAL_DIRS):
        ys, xs, yt, xt = _edge_slices(H, W, dy, dx)
        acc += (E[d, ys, xs][None] * (r[:, ys, xs] - r[:, yt, xt]) ** 2).sum()
    return float(acc)


def intensity(v: np.ndarray) -> np.ndarray:
    """|v| of Sec. 5.1 read as the channel mean (the reading under which the
    monochrome prior of Sec. 6.2 vanishes exactly for grey illumination)."""
    return (v[0] + v[1] + v[2]) / 3.0


def chromaticity(v: np.ndarray, p: OracleParams) -> np.ndarray:
    """C = v / |v| (Sec. 5.1); white where the intensity is below the floor."""
    m = intensity(v)
    ok = m >= p.chroma_floor
    safe = np.where(ok, m, 1.0)
    return np.where(ok[None], v / safe[None], 1.0)


def delta_chroma(C: np.ndarray) -> np.ndarray:
    """Delta C of Sec. 6.2: the largest chromaticity difference (L2 over channels)
    to any of the four in-image neighbours."""
    _, H, W = C.shape
    out = np.zeros((H, W))
    dx = np.sqrt(((C[:, :, 1:] - C[:, :, :-1]) ** 2).sum(axis=0))   # between x and x+1
    dy = np.sqrt(((C[:, 1:, :] - C[:, :-1, :]) ** 2).sum(axis=0))   # between y and y+1
    out[:, :-1] = np.maximum(out[:, :-1], dx)
    out[:, 1:] = np.maximum(out[:, 1:], dx)
    out[:-1, :] = np.maximum(out[:-1, :], dy)
    out[1:, :] = np.maximum(out[1:, :], dy)
    return out


def soft_retinex_weight(I: np.ndarray, p: OracleParams) -> np.ndarray:
    """w_SR = 1 - exp(-50 Delta C), per pixel (Sec. 6.2)."""
    return 1.0 - np.exp(-p.retinex_k * delta_chroma(chromaticity(I, p)))


@dataclass
class FrameData:
    """Everything about one frame that stays fixed while its unknowns change."""

    I: np.ndarray                      # (3, H, W)
    ids: np.ndarray                    # (H, W) int, colour index in [0, K)
    wsr: np.ndarray                    # (H, W)
    C: np.ndarray                      # (3, H, W) chromaticity of I
    gamma: Optional[np.ndarray] = None  # (9, H, W) 0/1 temporal pair gates (0 outside the image)
    rprev: Optional[np.ndarray] = None  # (9, 3, H, W) previous-frame r at each window pixel
    sp_edges: Optional[np.ndarray] = None  # (4, H, W) active spatial pairs (SPATIAL_DIRS), when on

    @property
    def shape(self):
        return self.I.shape[1:]


def prepare_frame(I: np.ndarray, ids: np.ndarray, p: OracleParams,
                  prev_C: Optional[np.ndarray] = None,
                  prev_r: Optional[np.ndarray] = None) -> FrameData:
    """Per-frame fixed data: chromaticity, soft-Retinex weight and, for video,
    the temporal-consistency pairs against the previous frame's final
    reflectance (Sec. 6.1)."""
    I = np.asarray(I, np.float64)
    C = chromaticity(I, p)
    wsr = 1.0 - np.exp(-p.retinex_k * delta_chroma(C))
    fd = FrameData(I=I, ids=np.asarray(ids).astype(np.int64), wsr=wsr, C=C)
    if p.spatial_pairs:
        fd.sp_edges = spatial_edges(C, p)
    if prev_C is not None:
        _, H, W = I.shape
        gamma = np.zeros((9, H, W))
        rprev = np.zeros((9, 3, H, W))
        for o, (dy, dx) in enumerate(WINDOW):
            for y in range(H):
                yy = y + dy
                if yy < 0 or yy >= H:
                    continue
                x0, x1 = max(0, -dx), min(W, W - dx)     # x + dx stays in [0, W)
                if x1 <= x0:
                    continue
                cp = prev_C[:, yy, x0 + dx:x1 + dx]
                d = np.sqrt(((C[:, y, x0:x1] - cp) ** 2).sum(axis=0))
                gamma[o, y, x0:x1] = (d < p.chroma_gate).astype(np.float64)
                rprev[o, :, y, x0:x1] = prev_r[:, yy, x0 + dx:x1 + dx]
        fd.gamma, fd.rprev = gamma, rprev
    return fd


def full_basis(b: np.ndarray) -> np.ndarray:
    """(K+1, 3) basis with the white illuminant b_0 = (1,1,1) first (Sec. 4)."""
    return np.vstack([np.ones((1, 3)), np.asarray(b, np.float64)])


def shading(T: np.ndarray, b: np.ndarray) -> np.ndarray:
    """S_c = sum_{k=0..K} b_{k,c} T_k (Sec. 4, eq. imageformation)."""
    B = full_basis(b)
    return np.einsum("kc,khw->chw", B, T)


def cluster_log_reflectance(b: np.ndarray, ids: np.ndarray) -> np.ndarray:
    """r_cluster = ln b_id (Sec. 5.1 and eq. clustering-term), (3, H, W)."""
    return np.log(np.asarray(b, np.float64))[ids].transpose(2, 0, 1)


def forward_diff(f: np.ndarray):
    """Forward differences along x and y of the last two axes; the difference at
    the last column / row does not exist (it is dropped, not padded)."""
    return f[..., :, 1:] - f[..., :, :-1], f[..., 1:, :] - f[..., :-1, :]


def rgrad_norm(r: np.ndarray) -> np.ndarray:
    """|grad r(x)|_2 over both directions and all three channels (eq.
    reflectance-sparsity-term), zero where no forward neighbour exists."""
    gx, gy = forward_diff(r)
    sq = np.zeros(r.shape[1:])
    sq[:, :-1] += (gx ** 2).sum(axis=0)
    sq[:-1, :] += (gy ** 2).sum(axis=0)
    return np.sqrt(sq)


def energy_terms(u: np.ndarray, b: np.ndarray, fd: FrameData, p: OracleParams) -> dict:
    """Each term of E_decomp (eq. giv-energy) at (u, b), summed over pixels.

    data       eq. data-term
    cluster    eq. clustering-term
    rsparsity  eq. reflectance-sparsity-term
    rconsist   spatio-temporal consistency prior (3x3 window reading), video only
    mono       soft-Retinex weighted monochromaticity prior, w_SR per pixel
    isparsity  eq. shading-sparsity-term
    smooth     eq. smoothness-term (l1 of the forward gradient of every layer)
    nonneg     eq. nonnegativityterm
    """
    u = np.asarray(u, np.float64)
    r, T = u[:3], u[3:]
    R = np.exp(r)
    S = shading(T, b)
    out = {}
    out["data"] = p.lam_data * ((fd.I - R * S) ** 2).sum()
    out["cluster"] = p.lam_cluster * ((r - cluster_log_reflectance(b, fd.ids)) ** 2).sum()
    out["rsparsity"] = p.lam_rsparsity * (rgrad_norm(r) ** p.p).sum()
    if fd.gamma is not None:
        acc = 0.0
        for o in range(9):
            acc += (fd.gamma[o] * ((r - fd.rprev[o]) ** 2).sum(axis=0)).sum()
        out["rconsist"] = p.lam_rconsistency * acc
    else:
        out["rconsist"] = 0.0
    if fd.sp_edges is not None:
        out["rconsist"] += p.lam_rconsistency * spatial_sq(r, fd.sp_edges)
    out["mono"] = p.lam_mono * (fd.wsr * ((S - intensity(S)[None]) ** 2).sum(axis=0)).sum()
    out["isparsity"] = p.lam_isparsity * np.abs(T[1:]).sum()
    gx, gy = forward_diff(T)
    out["smooth"] = p.lam_smooth * (np.abs(gx).sum() + np.abs(gy).sum())
    out["nonneg"] = p.lam_nonneg * np.maximum(-T, 0.0).sum()
    return out


def total_energy(u, b, fd: FrameData, p: OracleParams) -> float:
    return float(sum(energy_terms(u, b, fd, p).values()))
