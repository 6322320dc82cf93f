"""One weighted Gerchberg-Saxton (WGS) step around the compressed transforms.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper runs weighted GS (citing Kim et al. for the weighting) between the
spot-wise forward and adjoint transforms ("A Full-Field 2D Tweezer Array",
WGS paragraph; GS itself in "Aberration-Space Holography": nearfield and
farfield are corrected to the source and target amplitudes each iteration).
It prints no formula for the weights, so the classic weighted-GS update is
the reading taken here, step by step:

  1. f = A exp(i phi);  E = F_c f
  2. a_k = |E_k|
  3. r_k = (a_k / ||a||_2) / (t_k / ||t||_2)
  4. W_k <- W_k * r_k^(-p) where a_k > 0 (unchanged where a_k = 0);
     then W <- W / mean(W)
  5. y_k = W_k t_k E_k / a_k   (y_k = W_k t_k where a_k = 0)
  6. g = F_c^{-1} y
  7. phi <- atan2(Im g, Re g)    with atan2(0, 0) = 0

Variants (the same steps, a different farfield update):
  phase-fixed WGS (the weighted-GS reference the paper cites fixes the
  farfield phases after some iterations): step 5 uses stored phases psi_k,
  y_k = W_k t_k exp(i psi_k), from the iteration at which they were frozen;
  experimental feedback (the paper's software closes the loop on camera
  measurements): step 2 takes a_k from measured amplitudes instead of |E_k|
  (values <= 0 count as dark); the projection still uses arg E_k.

Figures of merit of the fields E of the step (standard WGS diagnostics, not
defined in the paper): efficiency eta = sum_k a_k^2 / (P * sum_x A^2);
with I_k = a_k^2 / t_k^2, uniformity 1 - (max I - min I)/(max I + min I)
and relative spread std(I)/mean(I); and sum_k a_k^2.
"""

import numpy as np

from .transform import forward, adjoint


def wgs_stats(E, t, amp):
    a2 = np.abs(E) ** 2
    t = np.asarray(t, dtype=np.float64)
    amp = np.asarray(amp, dtype=np.float64)
    P = amp.size
    denom = P * np.sum(amp ** 2)
    eta = np.sum(a2) / denom if denom > 0 else 0.0
    I = a2 / t ** 2
    mx, mn = np.max(I), np.min(I)
    unif = 1.0 - (mx - mn) / (mx + mn) if (mx + mn) > 0 else 0.0
    mu = np.mean(I)
    spread = np.std(I) / mu if mu > 0 else 0.0
    return np.array([eta, unif, spread, np.sum(a2)])


def wgs_farfield(E, weights, t, power=1.0, measured=None, fixed_phase=None):
    """Steps 2-5: the weight update and the farfield projection y of fields E
    (amplitudes from `measured` if given; phases `fixed_phase` if given).

    Returns (y, weights_new).
    """
    E = np.asarray(E, dtype=np.complex128)
    t = np.asarray(t, dtype=np.float64)
    W = np.asarray(weights, dtype=np.float64).copy()
    if measured is None:
        a = np.abs(E)
    else:
        a = np.maximum(np.asarray(measured, dtype=np.float64), 0.0)
    na = np.sqrt(np.sum(a ** 2))
    nt = np.sqrt(np.sum(t ** 2))
    lit = a > 0
    r = np.ones_like(a)
    if na > 0:
        r[lit] = (a[lit] / na) / (t[lit] / nt)
    W[lit] = W[lit] * r[lit] ** (-power)
    W = W / np.mean(W)

    if fixed_phase is not None:
        return W * t * np.exp(1j * np.asarray(fixed_phase, np.float64)), W
    y = W * t + 0j
    nz = np.abs(E) > 0
    y[nz] = W[nz] * t[nz] * E[nz] / np.abs(E[nz])
    return y, W


def wgs_step(phi, weights, t, amp, w, basis, geom, power=1.0, workers=None,
             measured=None, fixed_phase=None, return_y=False):
    """One WGS iteration. Returns (phi_new, weights_new, E, stats), and the
    farfield projection y (phi_new = arg F_c^{-1} y) last if return_y."""
    phi = np.asarray(phi, dtype=np.float64)
    amp = np.asarray(amp, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)

    f = amp * np.exp(1j * phi)
    E = forward(f, w, basis, geom, workers=workers)
    y, W = wgs_farfield(E, weights, t, power, measured, fixed_phase)
    g = adjoint(y, w, basis, geom, workers=workers)
    phi_new = np.arctan2(g.imag, g.real)
    if return_y:
        return phi_new, W, E, wgs_stats(E, t, amp), y
    return phi_new, W, E, wgs_stats(E, t, amp)


def wgs_run(phi0, t, amp, w, basis, geom, n_iter, power=1.0, workers=None,
            keep=(), fix_phase_after=0):
    """n_iter WGS steps from phi0 with W = 1; with fix_phase_after = n > 0
    the farfield phases arg E of iteration n - 1 are used from iteration n
    on.

    Returns (phi, W, E_last, stats[n_iter, 4], kept) where ``kept`` maps each
    iteration index listed in ``keep`` to the (phi, W) state entering it.
    """
    phi = np.asarray(phi0, dtype=np.float64)
    W = np.ones(np.asarray(t).shape[0])
    stats = np.zeros((n_iter, 4))
    kept = {}
    E = None
    psi = None
    for it in range(n_iter):
        if it in keep:
            kept[it] = (phi.copy(), W.copy())
        fixed = psi if (fix_phase_after > 0 and it >= fix_phase_after) else None
        phi, W, E, st = wgs_step(phi, W, t, amp, w, basis, geom, power,
                                 workers, fixed_phase=fixed)
        if fix_phase_after > 0 and it == fix_phase_after - 1:
            psi = np.angle(E)
        stats[it] = st
    return phi, W, E, stats, kept
