"""Parameters of the oracle (paper Sec. 8, "Parameters" paragraph, and Sec. 6).

The lambda values are the fixed set the paper uses for all its results.
epsilon for the non-negativity reweighting is the value given with that term
(Sec. 6.4.1).  The other constants are readings of passages that leave them open;
each is listed with its reasoning in the design notes.
"""
from __future__ import annotations

from dataclasses import dataclass, replace


@dataclass(frozen=True)
class OracleParams:
    # energy weights (Sec. 8 "Parameters")
    lam_data: float = 5000.0
    lam_cluster: float = 200.0
    lam_rsparsity: float = 20.0
    p: float = 1.0                 # exponent of the reflectance-gradient sparsity norm
    lam_rconsistency: float = 10.0
    lam_mono: float = 10.0
    lam_isparsity: float = 3.0
    lam_smooth: float = 3.0
    lam_nonneg: float = 1000.0
    lam_ir: float = 10.0           # base-colour intensity regulariser (Sec. 6.3)
    lam_cr: float = 100.0          # base-colour chromaticity regulariser (Sec. 6.3)
    # constants
    eps_nonneg: float = 0.002      # Sec. 6.4.1
    eps_irls: float = 0.002        # reading: the same epsilon guards the l_p IRLS weights
    retinex_k: float = 50.0        # soft-Retinex weight 1 - exp(-50 dC), Sec. 6.2
    chroma_gate: float = 0.1       # reading: temporal pairs count when |dC|_2 < 0.1
    chroma_floor: float = 1e-6     # reading: chromaticity is white below this intensity
    cr_mode: str = "chroma"        # "chroma" (anchored to the initial estimate) or "literal"
    # Scale of the data sum of the base-colour refinement energy (Sec. 6.3):
    # "pixel" divides it by the pixel count (the reading the solver uses by
    # default), "sum" takes the pixel sum as printed.
    bstep_scale: str = "pixel"
    # Storage precision of the unknowns between steps: "f64", or "f32" to round
    # them where a single-precision implementation stores them (the initial
    # state and after every layer step).  The discrete IRLS branches (T > 0 for
    # the non-negativity weight) are decided on the stored state, so an FP32
    # implementation is compared with the "f32" setting; all arithmetic stays FP64.
    state_precision: str = "f64"
    # Spatial pairs of the consistency prior (Sec. 6.1: every pixel is tied to
    # randomly sampled pixels of a small window under a chromaticity gate):
    # off by default; the reading and its seeded sampling are in energy.py.
    spatial_pairs: bool = False
    spatial_seed: int = 2019


def default_params(**kw) -> OracleParams:
    return replace(OracleParams(), **kw)
