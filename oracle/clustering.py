"""Base-colour initialisation by chromaticity clustering (Sec. 5.1), in float64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper clusters the first frame in a discretised chromaticity space: a
histogram of C(x) = I(x) / |I(x)| with 10 partitions per axis, weighted k-means
on the bin mid-points with the bin populations as weights and a user-given upper
bound K (10), centres closer than 0.2 merged (the smaller cluster into the
larger), every pixel assigned to its closest centre, and the mean RGB of each
cluster's pixels taken as its initial base colour.

Readings where the paper is silent (listed with the other readings in the
design notes):
  * |.| is the channel mean, so every chromaticity component lies in [0, 3]
    for a non-negative colour; the 10 partitions per axis cover [0, 3] with
    width 0.3 (component c of a pixel falls in partition floor(10 C_c / 3),
    clamped to 0..9); below the intensity floor a pixel is white (1, 1, 1).
  * k-means starts from the most populated bin and adds the non-empty bin
    farthest from the chosen centres (squared L2; ties to the lowest bin
    index), stopping early when every bin coincides with a centre; Lloyd
    iterations (bins to the nearest centre, ties to the lowest centre index;
    centres to the weighted mean of their bins, summed in bin order; a centre
    without bins stays) run until the assignment repeats, at most 100 times.
  * merging repeatedly takes the closest pair of centres (ties: the lowest
    index pair) while their L2 distance is below the threshold; the cluster
    with the smaller population (ties: the higher index) joins the other,
    whose centre becomes the weighted mean of the joint bins; the order of the
    remaining clusters is kept.
  * pixels go to the centre nearest to their own chromaticity (squared L2,
    ties to the lowest index); a cluster left without pixels is dropped and the
    pixels are assigned again.
Distances are formed as d0*d0 + d1*d1 + d2*d2, left to right, so that the
discrete decisions can be reproduced exactly in FP64.

For frames after the first, `nearest_ids` assigns pixels to the base colour
whose chromaticity is nearest (the same rule against the current colours).
"""
from __future__ import annotations

import numpy as np

from .energy import chromaticity
from .params import OracleParams

BINS = 10
C_MAX = 3.0
MAX_LLOYD = 100


def bin_coords(C: np.ndarray) -> np.ndarray:
    """(3, ...) integer partition index of every chromaticity component."""
    j = np.floor(C * float(BINS) / C_MAX)
    return np.clip(j, 0, BINS - 1).astype(np.int64)


def chroma_histogram(I: np.ndarray, p: OracleParams) -> np.ndarray:
    """Pixel count of each of the BINS^3 bins, flat index (j0 * BINS + j1) * BINS + j2."""
    C = chromaticity(np.asarray(I, np.float64), p)
    j = bin_coords(C).reshape(3, -1)
    flat = (j[0] * BINS + j[1]) * BINS + j[2]
    return np.bincount(flat, minlength=BINS ** 3).astype(np.int64)


def bin_midpoint(b: int) -> np.ndarray:
    j = (b // (BINS * BINS), (b // BINS) % BINS, b % BINS)
    return np.array([(jc + 0.5) * C_MAX / BINS for jc in j])


def _d2(a, b) -> float:
    d0, d1, d2 = a[0] - b[0], a[1] - b[1], a[2] - b[2]
    return d0 * d0 + d1 * d1 + d2 * d2


def _weighted_mean(bins, hist):
    s = np.zeros(3)
    w = 0
    for b in bins:
        s = s + float(hist[b]) * bin_midpoint(b)
        w += int(hist[b])
    return s / float(w)


def kmeans_seeds(hist: np.ndarray, K: int) -> list:
    """Farthest-point seeds: bin indices of the chosen starting centres."""
    nz = [int(b) for b in np.flatnonzero(hist)]
    if not nz:
        return []
    first = max(nz, key=lambda b: (hist[b], -b))      # most populated, lowest index on ties
    seeds = [first]
    while len(seeds) < K:
        best, best_d = None, 0.0
        for b in nz:
            d = min(_d2(bin_midpoint(b), bin_midpoint(s)) for s in seeds)
            if d > best_d:
                best, best_d = b, d
        if best is None:
            break
        seeds.append(best)
    return seeds


def weighted_kmeans(hist: np.ndarray, K: int):
    """Centres (k, 3) and the cluster of every non-empty bin {bin: cluster}."""
    nz = [int(b) for b in np.flatnonzero(hist)]
    centres = [bin_midpoint(s) for s in kmeans_seeds(hist, K)]
    assign = None
    for _ in range(MAX_LLOYD):
        new = {}
        for b in nz:
            m = bin_midpoint(b)
            dists = [_d2(m, c) for c in centres]
            new[b] = int(np.argmin(dists))            # first minimum: lowest centre index
        if new == assign:
            break
        assign = new
        for j in range(len(centres)):
            members = [b for b in nz if assign[b] == j]
            if members:
                centres[j] = _weighted_mean(members, hist)
    return np.array(centres), assign


def merge_clusters(centres: np.ndarray, assign: dict, hist: np.ndarray, threshold: float):
    """Merge centres closer than threshold; returns (centres, assign) renumbered."""
    centres = [np.asarray(c, np.float64) for c in centres]
    members = [[b for b in sorted(assign) if assign[b] == j] for j in range(len(centres))]
    while True:
        pair, best = None, None
        for a in range(len(centres)):
            for b in range(a + 1, len(centres)):
                d = np.sqrt(_d2(centres[a], centres[b]))
                if d < threshold and (best is None or d < best):
                    pair, best = (a, b), d
        if pair is None:
            break
        a, b = pair
        wa = sum(int(hist[x]) for x in members[a])
        wb = sum(int(hist[x]) for x in members[b])
        keep, drop = (a, b) if wa >= wb else (b, a)
        members[keep] = sorted(members[keep] + members[drop])
        if members[keep]:
            centres[keep] = _weighted_mean(members[keep], hist)
        del centres[drop], members[drop]
    out = {}
    for j, ms in enumerate(members):
        for x in ms:
            out[x] = j
    return np.array(centres), out


def assign_pixels(I: np.ndarray, centres: np.ndarray, p: OracleParams) -> np.ndarray:
    """Index of the centre nearest to every pixel's chromaticity (ties: lowest)."""
    C = chromaticity(np.asarray(I, np.float64), p)
    best = np.full(C.shape[1:], np.inf)
    ids = np.zeros(C.shape[1:], np.int64)
    for j, c in enumerate(centres):
        d0, d1, d2 = C[0] - c[0], C[1] - c[1], C[2] - c[2]
        d = d0 * d0 + d1 * d1 + d2 * d2
        closer = d < best
        best = np.where(closer, d, best)
        ids = np.where(closer, j, ids)
    return ids


def cluster_frame(I: np.ndarray, K_max: int, p: OracleParams, merge_threshold: float = 0.2):
    """The whole Sec. 5.1 initialisation: (ids (H, W) uint8, colours (k, 3), centres (k, 3))."""
    I = np.asarray(I, np.float64)
    hist = chroma_histogram(I, p)
    centres, assign = weighted_kmeans(hist, K_max)
    centres, assign = merge_clusters(centres, assign, hist, merge_threshold)
    while True:
        ids = assign_pixels(I, centres, p)
        counts = np.bincount(ids.ravel(), minlength=len(centres))
        if np.all(counts > 0):
            break
        centres = centres[counts > 0]
    colours = np.zeros((len(centres), 3))
    for j in range(len(centres)):
        m = ids == j
        for c in range(3):
            colours[j, c] = I[c][m].sum() / m.sum()
    return ids.astype(np.uint8), colours, centres


def nearest_ids(I: np.ndarray, b: np.ndarray, p: OracleParams) -> np.ndarray:
    """Cluster ids of a later frame: the base colour of nearest chromaticity."""
    Cb = chromaticity(np.asarray(b, np.float64).T[:, :, None], p)[:, :, 0].T    # (K, 3)
    return assign_pixels(I, Cb, p).astype(np.uint8)
