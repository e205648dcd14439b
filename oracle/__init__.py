"""FP64 CPU oracle for the global-illumination decomposition solver.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, deliberately
unoptimised restatement of the method of "Real-Time Global Illumination
Decomposition of Videos" (Meka et al.): the energy of Sec. 6, the IRLS
reweighting of Sec. 6.4 and the alternating Gauss-Newton / PCG solve of Sec. 7.
It exists to check the GPU library.  Only the test-suite, the smoke check and
the CPU-baseline leg of the benchmark may import it; the product path never
does, and it shares no code with the HIP kernels or their binding.

Everything is NumPy/SciPy in float64.  Modules:
  params     -- the paper's parameter set and the readings of unclear passages
  energy     -- chromaticity, soft-Retinex weight, temporal window, true energy
  gauss_newton -- IRLS weights, matrix-free J^T J, right-hand side, Jacobi PCG
  explicit   -- row-by-row residual vector and sparse Jacobian, direct solve
  basecolor  -- the base-colour (B-)step normal equations and SVD solve
  schedule   -- initialisation, the per-frame alternating schedule, video loop
  clustering -- base-colour initialisation by chromaticity clustering (Sec. 5.1)
"""
from .params import OracleParams, default_params
from .energy import (FrameData, prepare_frame, energy_terms, total_energy, chromaticity,
                     delta_chroma, soft_retinex_weight)
from .gauss_newton import (Linearisation, linearise, apply_normal, rhs, jacobi_diag, pcg,
                           surrogate_energy)
from .explicit import assemble_residuals, direct_step
from .basecolor import bstep_sums, bstep_system, bstep_solve
from .schedule import init_state, decompose_frame, decompose_clip, FrameResult
from .clustering import cluster_frame, nearest_ids

__all__ = [
    "OracleParams", "default_params", "FrameData", "prepare_frame", "energy_terms",
    "total_energy", "chromaticity", "delta_chroma", "soft_retinex_weight", "Linearisation",
    "linearise", "apply_normal", "rhs", "jacobi_diag", "pcg", "surrogate_energy",
    "assemble_residuals", "direct_step", "bstep_sums", "bstep_system", "bstep_solve",
    "init_state", "decompose_frame", "decompose_clip", "FrameResult", "cluster_frame", "nearest_ids",
]
