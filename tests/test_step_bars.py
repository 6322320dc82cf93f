"""The staged WGS-step bars (tests/tolerance.py) are bounds: perturbing the
oracle's fields by errors of FP32 size, in FP64 on the CPU, moves the
oracle's weights and phases by less than the bars derived from those
perturbations, including the ill-conditioned first step from a random phase
with many spots."""

import numpy as np
import pytest

import oracle
from tolerance import step_bars, derived_phase_bar, wrap, STEP_PHASE_MASK


@pytest.mark.parametrize("N,scale,seed", [(2500, 1e-5, 1), (2500, 1e-4, 2),
                                          (400, 1e-5, 3)])
def test_step_bars_bound_perturbed_steps(N, scale, seed):
    nx, ny = 96, 64
    modes = [1, 2, 3, 4, 5]
    rng = np.random.default_rng(seed)
    geom = oracle.Geometry(nx, ny)
    basis = oracle.ZernikeBasis(modes)
    w = rng.normal(0, 0.4, size=(N, len(modes)))
    w[:, 0] = np.pi * rng.uniform(-ny / 2, ny / 2, N) * geom.R / ny
    w[:, 1] = np.pi * rng.uniform(-nx / 2, nx / 2, N) * geom.R / nx
    t = rng.uniform(0.5, 1.0, N)
    amp = rng.uniform(0.2, 1.0, (ny, nx))
    phi = rng.uniform(-np.pi, np.pi, (ny, nx))
    E = oracle.forward(amp * np.exp(1j * phi), w, basis, geom)
    y, W = oracle.wgs_farfield(E, np.ones(N), t)
    g = oracle.adjoint(y, w, basis, geom).reshape(-1)
    rms = np.sqrt(np.mean(np.abs(E) ** 2))
    # an error of the FP32 kind: independent per spot, of size
    # scale * max(|E|, rms)
    dE = scale * np.maximum(np.abs(E), rms) * (rng.normal(size=N) + 1j * rng.normal(size=N)) / 2
    y2, W2 = oracle.wgs_farfield(E + dE, np.ones(N), t)
    g2 = oracle.adjoint(y2, w, basis, geom).reshape(-1)
    wb, sigma = step_bars(E, dE, W, t)
    assert np.all(np.abs(W2 - W) / W <= wb)
    # the farfield error is within its bound spot by spot
    assert np.all(np.abs(y2 - y) <= W * t * (wb + np.abs(dE) / np.abs(E)) * 1.001)
    keep = np.abs(g) >= STEP_PHASE_MASK * np.sqrt(np.mean(np.abs(g) ** 2))
    dphi = np.abs(wrap(np.angle(g2) - np.angle(g)))
    bar = derived_phase_bar(g, sigma, rel_adj=0.0)
    ratio = dphi[keep] / bar[keep]
    assert ratio.max() <= 1.0
    # and it is a useful bound, not a vacuous one: the largest error
    # reaches a sizeable part of it
    assert ratio.max() >= 0.02
