"""Seeded synthetic inputs (frames, cluster ids, initial base colours, ground truth)."""
from .generator import (Clip, make_clip, downsample_clip, workload_clip, mixed_batch_specs,
                        WORKLOADS, MIXED_SIZES)

__all__ = ["Clip", "make_clip", "downsample_clip", "workload_clip", "mixed_batch_specs",
           "WORKLOADS", "MIXED_SIZES"]
