"""Initialisation and the alternating schedule (Sec. 7.1, sparse-dense splitting).

One frame is G outer iterations; each is a layer step (one IRLS Gauss-Newton
step whose normal equations get P PCG iterations) followed, when refinement is
active, by a base-colour step.  The energy is recorded after each half-step.
Video frames after the first start from the previous frame's final layers and
base colours; the temporal-consistency prior then ties r to the previous frame's
final r.

Initialisation of the first frame (the paper initialises R from the clustered
reflectance, Sec. 5.1; the illumination start is a reading):
  r = ln b_id,  T_0 = clip(|I| / |R|, 0, 4),  T_k = 0.01 for k >= 1.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np

from .basecolor import bstep
from .clustering import nearest_ids
from .energy import FrameData, cluster_log_reflectance, intensity, prepare_frame, total_energy
from .explicit import direct_step
from .gauss_newton import linearise, pcg
from .params import OracleParams


def store(u: np.ndarray, p: OracleParams) -> np.ndarray:
    """The unknowns as stored between steps (see OracleParams.state_precision)."""
    if p.state_precision == "f32":
        return np.asarray(u, np.float32).astype(np.float64)
    return u


def init_state(I: np.ndarray, ids: np.ndarray, b: np.ndarray) -> np.ndarray:
    I = np.asarray(I, np.float64)
    K = np.asarray(b).shape[0]
    H, W = I.shape[1:]
    rcl = cluster_log_reflectance(b, np.asarray(ids).astype(np.int64))
    u = np.empty((K + 4, H, W))
    u[:3] = rcl
    u[3] = np.clip(intensity(I) / intensity(np.exp(rcl)), 0.0, 4.0)
    u[4:] = 0.01
    return u


@dataclass
class FrameResult:
    u: np.ndarray
    b: np.ndarray
    energy: float
    energies: list = field(default_factory=list)   # (label, E) after each half-step
    pcg: list = field(default_factory=list)        # per layer step: {"rz", "iters"}
    fd: Optional[FrameData] = None
    starts: list = field(default_factory=list)     # unknowns at the start of every GN step (keep_starts)


def decompose_frame(I, ids, b, b_init, p: OracleParams, G: int, P: int, *, u0=None,
                    prev=None, refine: bool = True, solver: str = "pcg",
                    record: bool = True, keep_starts: bool = False) -> FrameResult:
    """Run the fixed schedule on one frame.

    prev: (C_prev, r_prev) of the previous frame for the temporal prior, or None.
    solver: "pcg" (P Jacobi-PCG iterations) or "direct" (exact normal-equation solve).
    ids None: every pixel takes the base colour of nearest chromaticity at the
    frame's start (the assignment rule of Sec. 5.1 against the current colours).
    """
    b = np.asarray(b, np.float64).copy()
    if ids is None:
        ids = nearest_ids(I, b, p)
    fd = prepare_frame(I, ids, p, *(prev if prev is not None else (None, None)))
    u = store(init_state(fd.I, fd.ids, b), p) if u0 is None else np.asarray(u0, np.float64).copy()
    energies, infos, starts = [], [], []
    for _ in range(G):
        if keep_starts:
            starts.append(u.copy())
        lin = linearise(u, b, fd, p)
        if solver == "pcg":
            delta, info = pcg(lin, P)
        elif solver == "direct":
            delta, info = direct_step(lin), {"rz": float("nan"), "iters": -1}
        else:
            raise ValueError(solver)
        u = store(u + delta, p)
        infos.append(info)
        if record:
            energies.append(("T", total_energy(u, b, fd, p)))
        if refine:
            b, _ok = bstep(u, b, b_init, fd.I, p)
            if record:
                energies.append(("B", total_energy(u, b, fd, p)))
    E = energies[-1][1] if (record and energies) else total_energy(u, b, fd, p)
    return FrameResult(u=u, b=b, energy=E, energies=energies, pcg=infos, fd=fd, starts=starts)


def decompose_clip(frames, ids, b_init, p: OracleParams, G: int, P: int, *, temporal: bool = True,
                   refine_mode: str = "every", solver: str = "pcg", nframes: int | None = None,
                   record: bool = True, keep_starts: bool = False):
    """Decompose frames in order with warm starts; returns the list of FrameResult.

    refine_mode: "every" (B-step in every outer iteration of every frame),
                 "first" (only on the first frame, as in the paper's timing run) or "off".
    """
    F = len(frames) if nframes is None else nframes
    b = np.asarray(b_init, np.float64).copy()
    u = None
    prev = None
    out = []
    for t in range(F):
        refine = refine_mode == "every" or (refine_mode == "first" and t == 0)
        res = decompose_frame(frames[t], None if ids is None or ids[t] is None else ids[t], b, b_init, p, G, P, u0=u,
                              prev=prev if temporal else None, refine=refine, solver=solver,
                              record=record, keep_starts=keep_starts)
        out.append(res)
        u, b = res.u, res.b
        prev = (res.fd.C, u[:3].copy())
    return out
