"""In-silico spot quality: the windowed Strehl proxy of the paper's metrology.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Methods, "Relative Strehl Metrology": for a camera image I, the quality of a
spot is S' = max I / sum I over a 21 x 21 pixel box around the spot (the box
is several times the diffraction-limited waist); dividing by the largest S'
gives the relative Strehl ratio.

In silico the "image" near spot k is the farfield intensity of the hologram
at win x win points around the spot, sampled every `step` DFT bins: each
point is a kernel with spot k's coefficients and its tilts moved by the
offset, i.e. the forward transform with an expanded spot list.  Here the
tilt coefficients are moved by pi * step * R / nx (x) and pi * step * R / ny
(y) per camera pixel, the slope of one bin for the orthonormal tilts
Z_2 = 2 xh and Z_1 = 2 yh.
"""

import numpy as np

from .transform import forward


def window_coefficients(w, ix, iy, dwx, dwy, win):
    """Coefficients of the win x win window points of every spot, spot-major
    with the window's x offset fastest: row (k * win + b) * win + a has
    w[k, ix] + (a - win // 2) dwx and w[k, iy] + (b - win // 2) dwy."""
    w = np.asarray(w, dtype=np.float64)
    N = w.shape[0]
    h = win // 2
    out = np.repeat(w, win * win, axis=0).reshape(N, win, win, -1)
    for b in range(win):
        for a in range(win):
            out[:, b, a, ix] += (a - h) * dwx
            out[:, b, a, iy] += (b - h) * dwy
    return out.reshape(N * win * win, -1)


def window_spacing(geom, step):
    """Coefficient changes (dwx, dwy) in radians that move a spot by `step`
    DFT bins along x and y: one bin is a phase slope of 2 pi / n per pixel,
    and the orthonormal tilts 2 xh, 2 yh have slope 2 / R per unit
    coefficient."""
    return np.pi * step * geom.R / geom.nx, np.pi * step * geom.R / geom.ny


def window_strehl(E, N, win):
    """S'_k = max |E|^2 / sum |E|^2 over spot k's window (0 for a dark one)."""
    I = np.abs(np.asarray(E, dtype=np.complex128)).reshape(N, win * win) ** 2
    tot = I.sum(axis=1)
    return np.where(tot > 0, I.max(axis=1) / np.where(tot > 0, tot, 1.0), 0.0)


def spot_quality(f, w, basis, geom, ix, iy, win=21, step=0.25, spots=None,
                 workers=None):
    """S' of the windows around the spots (all, or the subset `spots`)."""
    w = np.asarray(w, dtype=np.float64)
    if spots is not None:
        w = w[np.asarray(spots)]
    dwx, dwy = window_spacing(geom, step)
    ww = window_coefficients(w, ix, iy, dwx, dwy, win)
    E = forward(f, ww, basis, geom, workers=workers)
    return window_strehl(E, w.shape[0], win)
