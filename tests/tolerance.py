"""Parity bars between the FP32 HIP path and the FP64 oracle.

Spot and pixel fields: per element |d| <= rel * max(|ref|, rms(ref)) and
normwise ||d|| / ||ref|| <= rel, rel = 1e-4.  The rms floor keeps dark
outputs (whose relative error is inflated by the FP32 rounding of the other
terms of their sum) from failing a bar meant for typical outputs.
Phases: |wrap(phi - phi_ref)| <= 1e-3 rad on pixels whose reference
field magnitude is at least 1e-2 of the rms magnitude (arg is
well-conditioned there: its error is about |dg| / |g|).  For a whole WGS
step the farfield projection y = W t E/|E| also carries the forward's
relative error eps_E (~1e-5) into g, so |dg| ~ eps_E rms|g| and the same
1e-3 rad bar is applied where |g| >= 5e-2 rms|g| (about 0.25% of pixels of
a Rayleigh-distributed field are excluded; the excluded fraction and the
all-pixel max / rms errors are reported).
"""

import numpy as np

FIELD_REL = 1e-4
PHASE_RAD = 1e-3
PHASE_MASK = 1e-2
STEP_PHASE_MASK = 5e-2


def field_errors(got, ref):
    got = np.asarray(got, dtype=np.complex128).reshape(-1)
    ref = np.asarray(ref, dtype=np.complex128).reshape(-1)
    d = np.abs(got - ref)
    rms = np.sqrt(np.mean(np.abs(ref) ** 2))
    scale = np.maximum(np.abs(ref), rms)
    per = d / np.where(scale > 0, scale, 1.0)
    norm = np.linalg.norm(got - ref) / max(np.linalg.norm(ref), 1e-300)
    return float(per.max()), float(norm)


def assert_fields(got, ref, rel=FIELD_REL, what="field"):
    per, norm = field_errors(got, ref)
    assert per <= rel and norm <= rel, \
        "%s: max elementwise %.3e, normwise %.3e (bar %.1e)" % (what, per, norm, rel)
    return per, norm


def wrap(d):
    return np.angle(np.exp(1j * np.asarray(d, dtype=np.float64)))


def phase_errors(got, ref_phase, ref_field, mask=PHASE_MASK):
    ref_field = np.asarray(ref_field).reshape(-1)
    d = np.abs(wrap(np.asarray(got, np.float64).reshape(-1)
                    - np.asarray(ref_phase, np.float64).reshape(-1)))
    mag = np.abs(ref_field)
    rms = np.sqrt(np.mean(mag ** 2))
    keep = mag >= mask * rms
    return float(d[keep].max()) if keep.any() else 0.0, float(1 - keep.mean()), \
        float(d.max()), float(np.sqrt(np.mean(d ** 2)))


def assert_phase(got, ref_phase, ref_field, bar=PHASE_RAD, what="phase",
                 mask=PHASE_MASK):
    mx, excl, mx_all, rms_all = phase_errors(got, ref_phase, ref_field, mask)
    assert mx <= bar, "%s: max %.3e rad on well-conditioned pixels (bar %.1e); " \
        "excluded %.4f, all-pixel max %.3e rms %.3e" % (what, mx, bar, excl, mx_all, rms_all)
    return mx, excl, mx_all, rms_all


# Phase gradients: the field bar (elementwise with the rms floor, and
# normwise) against the FP64 analytic gradient; against FP64 central
# differences (truncation ~h^2, h = 1e-4 rad) |d| <= 1e-3 rms(grad_FD).
GRAD_REL = 1e-4
GRAD_FD_REL = 1e-3

