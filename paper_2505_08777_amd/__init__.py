"""Aberration-space holography hot path on MI355X (gfx950).

Per-spot propagation kernels exp(-i sum_d w_d^(n) Z_d(x)) merged into one
SLM hologram: the compressed forward/adjoint transforms and the weighted
Gerchberg-Saxton loop, as hand-written HIP kernels behind a C ABI
(include/ash.h).  This package is the thin Python binding.
"""

from ._lib import (AshError, INJECT_ALLOC, INJECT_BARRIER, LIB_PATH,
                   inject_failure, lib)
from .basis import principal_modes, zernike_monomials, zernike_table
from .context import (Batch, Context, Propagate, PropagateSpots, propagate,
                      spot_quality, window_coefficients)

__all__ = ["AshError", "Batch", "Context", "INJECT_ALLOC", "INJECT_BARRIER",
           "LIB_PATH", "Propagate",
           "PropagateSpots", "lib",
           "inject_failure", "principal_modes", "propagate", "spot_quality",
           "window_coefficients", "zernike_monomials", "zernike_table"]
