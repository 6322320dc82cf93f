"""One GPU WGS step against the FP64 oracle's step from the same state,
judged in stages (see tests/tolerance.py): the forward fields at the field
bar, the new weights at the bar the field errors imply through the weight
update, and the new phases (all pixels or a sample) at the bar the
farfield errors imply through the adjoint, never looser than the plain
bars where the step is well conditioned."""

import sys

import numpy as np

import oracle
from tolerance import (assert_fields, field_errors, step_bars,
                       assert_step_weights, assert_step_phase)


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def reference_step(phi, W, t, amp, w, basis, geom, pixels=None,
                   measured=None, fixed_phase=None, workers=None):
    """The oracle's step from (phi, W): fields E, new weights W', the
    farfield projection y and the adjoint g of y at `pixels` (all if None,
    flattened)."""
    f = np.asarray(amp, np.float64) * np.exp(1j * np.asarray(phi, np.float64))
    E = oracle.forward(f, w, basis, geom, workers=workers)
    y, W1 = oracle.wgs_farfield(E, W, t, measured=measured,
                                fixed_phase=fixed_phase)
    g = oracle.adjoint(y, w, basis, geom, pixels=pixels, workers=workers)
    return E, W1, y, np.asarray(g).reshape(-1)


def check_step(what, ph_gpu, W_gpu, E_gpu, ref, t, pixels=None,
               weights_from_fields=True, dpsi=None):
    """Stages 1-3 for GPU outputs (torch tensors or arrays) against
    reference_step's output; returns the per-stage figures."""
    E_ref, W_ref, y_ref, g_ref = ref
    E = np.asarray(E_gpu.cpu().numpy() if hasattr(E_gpu, "cpu") else E_gpu)
    W = np.asarray(W_gpu.cpu().numpy() if hasattr(W_gpu, "cpu") else W_gpu)
    ph = np.asarray(ph_gpu.cpu().numpy() if hasattr(ph_gpu, "cpu") else ph_gpu)
    ph = ph.reshape(-1)
    if pixels is not None:
        ph = ph[np.asarray(pixels)]
    fe = assert_fields(E, E_ref, what=what + " fields")
    dE = E.astype(np.complex128) - E_ref
    wb, sigma = step_bars(E_ref, dE, W_ref, t,
                          weights_from_fields=weights_from_fields, dpsi=dpsi)
    we = assert_step_weights(W, W_ref, wb, what=what + " weights")
    pe = assert_step_phase(ph, np.angle(g_ref), g_ref, sigma,
                           what=what + " phase")
    _say("  %s: fields %.2e/%.2e; weights max rel %.2e (bar up to %.2e, "
         "%.2f of it); phase max %.2e rad (%.2f of its bar, median derived "
         "bar %.2e, excluded %.4f)" % ((what,) + fe + we + pe))
    return {"fields": fe, "weights": we, "phase": pe,
            "abs_dE": np.abs(dE)}
