"""MI355X (gfx950) solver for the global-illumination decomposition of videos.

The solve runs in libgid.so (HIP kernels behind the C ABI of include/gid.h);
this package holds its sources (csrc/), the build script and a thin ctypes
binding (gid.py).
"""
from .gid import (Batch, GidError, Net, GidFrameStats, GidParams, KERNEL_KINDS, LIB_PATH, SIGNATURES, Solver, TERMS,
                  cluster_frame, correct_region, default_params, load_library, resynthesize)

__all__ = ["Batch", "GidError", "Net", "GidFrameStats", "GidParams", "KERNEL_KINDS", "LIB_PATH", "SIGNATURES", "Solver", "TERMS",
           "cluster_frame", "correct_region", "default_params", "load_library", "resynthesize"]
