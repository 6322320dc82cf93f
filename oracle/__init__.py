"""FP64 CPU oracle for aberration-space holography.

TEST INFRASTRUCTURE ONLY.  Nothing in the product package imports, links or
executes this package; only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may call it.  It shares no code with the
HIP path (``paper_2505_08777_amd``): the basis here is evaluated with the
Zernike radial formula in polar coordinates, the transforms are the plain
direct sums written with numpy, and every quantity is float64 / complex128.

Modules
-------
zernike    ANSI / Noll indexing and the radial-formula Zernike polynomials
           ("Aberration-Space Holography", the modal-expansion paragraph).
transform  compressed forward and adjoint transforms F_c, F_c^{-1} with
           per-spot kernels K_n(x) = exp(-i sum_d w_d^(n) Z_d(x))
           ("Aberration-Space Holography", compressed-sum equations).
wgs        one weighted Gerchberg-Saxton step ("A Full-Field 2D Tweezer
           Array", the WGS paragraph; the weighting is a stated reading).
grad       spot-amplitude loss with phase-gradient TV, its analytic phase
           gradient, central finite differences and the Adam update of the
           phase (Methods, "Computational Scaling", gradient-descent
           paragraph; Adam as published by Kingma and Ba); the basis
           moments of the forward and the gradient with respect to the
           kernel coefficients w.
quality    in-silico spot quality: the windowed Strehl proxy S' (Methods,
           "Relative Strehl Metrology") of farfield windows around spots.
principal  principal isoplanatic modes: the SVD rotation of the non-linear
           modes and its rank-K truncation (Methods, "Anisoplanatic
           Singular Value Decomposition").

Parity status: every function here is pinned by a ``-m "not gpu"`` test in
``tests/test_oracle_pins.py`` except the multi-step WGS trajectory, whose
FP32-vs-FP64 drift makes it "parity unpinned" beyond one step.
"""

from .zernike import (ansi_to_nm, nm_to_ansi, noll_to_nm, noll_to_ansi,
                      zernike_nm, ZernikeBasis, MonomialBasis)
from .transform import Geometry, kernel_phase, forward, adjoint
from .wgs import wgs_farfield, wgs_step, wgs_run, wgs_stats
from .grad import (spot_norm, spot_loss, tv_loss, total_loss, loss_grad,
                   fd_grad, adam_step, adam_run, forward_moments, coef_grad)
from .principal import linear_modes, RotatedBasis, principal_modes
from .quality import (window_coefficients, window_spacing, window_strehl,
                      spot_quality)

__all__ = [
    "ansi_to_nm", "nm_to_ansi", "noll_to_nm", "noll_to_ansi", "zernike_nm",
    "ZernikeBasis", "MonomialBasis", "Geometry", "kernel_phase", "forward",
    "adjoint", "wgs_farfield", "wgs_step", "wgs_run", "wgs_stats", "spot_norm", "spot_loss",
    "tv_loss", "total_loss", "loss_grad", "fd_grad", "adam_step", "adam_run",
    "linear_modes", "RotatedBasis", "principal_modes", "forward_moments",
    "coef_grad", "window_coefficients", "window_spacing", "window_strehl", "spot_quality",
]
