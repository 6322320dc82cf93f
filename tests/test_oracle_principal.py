"""Pins for the oracle's principal isoplanatic modes (SVD rotation).

Each check is fixed by the mathematics of the decomposition, not by the
oracle's own code: a matrix built with a known spectrum, exactness on
matrices of rank K, Eckart-Young's truncation error, the Cauchy-Schwarz
bound on the phase change and the direction of a rank-one matrix.
"""

import numpy as np
import pytest

import oracle

MODES = [1, 2, 3, 4, 5, 6, 7, 8, 9, 12]       # tilts + 8 aberration modes


def _geom_idx(nx=32, ny=24):
    geom = oracle.Geometry(nx, ny)
    return geom, np.arange(geom.P)


def _orth(rng, n, k):
    q, _ = np.linalg.qr(rng.normal(size=(n, k)))
    return q


def _w_with_block(rng, N, WR):
    w = np.zeros((N, len(MODES)))
    w[:, 0] = rng.uniform(-30, 30, N)
    w[:, 1] = rng.uniform(-30, 30, N)
    w[:, 2:] = WR
    return w


def test_linear_mode_classification():
    assert list(oracle.linear_modes(oracle.ZernikeBasis([0, 1, 2, 3, 4, 12]))) == \
        [True, True, True, False, False, False]
    mb = oracle.MonomialBasis([(0, 0), (1, 0), (0, 1), (2, 0)],
                              [[1, 0, 0, 0], [0, 2, 1, 0], [0, 1, 0, 3], [0, 0, 0, 0]])
    assert list(oracle.linear_modes(mb)) == [True, True, False, True]


def test_known_spectrum_and_eckart_young():
    rng = np.random.default_rng(1)
    N = 40
    s = np.array([9.0, 5.0, 3.0, 2.0, 1.0, 0.5, 0.25, 0.125])
    WR = _orth(rng, N, 8) @ np.diag(s) @ _orth(rng, 8, 8).T
    w = _w_with_block(rng, N, WR)
    basis = oracle.ZernikeBasis(MODES)
    for K in range(9):
        wK, bK, sigma = oracle.principal_modes(w, basis, K)
        np.testing.assert_allclose(sigma, s, rtol=1e-12)
        VK = bK.V
        np.testing.assert_allclose(VK.T @ VK, np.eye(K), atol=1e-12)
        resid = WR - WR @ VK @ VK.T
        np.testing.assert_allclose(np.sum(resid ** 2), np.sum(s[K:] ** 2),
                                   rtol=1e-10, atol=1e-24)
        # the new coefficient columns are orthogonal with norms sigma_j
        C = wK[:, 2:]
        np.testing.assert_allclose(C.T @ C, np.diag(s[:K] ** 2), atol=1e-10)
        # linear modes pass through untouched
        np.testing.assert_array_equal(wK[:, :2], w[:, :2])
        assert bK.D == 2 + K


def test_rank_k_matrix_is_exact():
    rng = np.random.default_rng(2)
    N, K = 30, 3
    WR = rng.normal(size=(N, K)) @ rng.normal(size=(K, 8))
    w = _w_with_block(rng, N, WR)
    basis = oracle.ZernikeBasis(MODES)
    geom, idx = _geom_idx()
    th = oracle.kernel_phase(w, basis, geom, idx)
    wK, bK, sigma = oracle.principal_modes(w, basis, K)
    assert np.all(sigma[K:] < 1e-12 * sigma[0])
    thK = oracle.kernel_phase(wK, bK, geom, idx)
    assert np.max(np.abs(thK - th)) < 1e-11
    f = rng.normal(size=geom.P) + 1j * rng.normal(size=geom.P)
    E = oracle.forward(f, w, basis, geom)
    EK = oracle.forward(f, wK, bK, geom)
    assert np.max(np.abs(EK - E)) < 1e-10 * np.max(np.abs(E))


def test_full_rank_keeps_phases_and_k0_keeps_linear_part():
    rng = np.random.default_rng(3)
    N = 25
    w = _w_with_block(rng, N, rng.normal(0, 1.0, size=(N, 8)))
    basis = oracle.ZernikeBasis(MODES)
    geom, idx = _geom_idx(20, 16)
    th = oracle.kernel_phase(w, basis, geom, idx)
    w8, b8, _ = oracle.principal_modes(w, basis, 8)
    assert np.max(np.abs(oracle.kernel_phase(w8, b8, geom, idx) - th)) < 1e-11
    w0, b0, _ = oracle.principal_modes(w, basis, 0)
    lin = oracle.kernel_phase(w[:, :2], oracle.ZernikeBasis(MODES[:2]), geom, idx)
    assert np.max(np.abs(oracle.kernel_phase(w0, b0, geom, idx) - lin)) < 1e-11


def test_phase_change_within_cauchy_schwarz_bound():
    rng = np.random.default_rng(4)
    N = 50
    w = _w_with_block(rng, N, rng.normal(0, 1.0, size=(N, 8)))
    basis = oracle.ZernikeBasis(MODES)
    geom, idx = _geom_idx(24, 24)
    xh, yh = geom.coords(idx)
    ZR = basis.evaluate(xh, yh)[2:]                       # [8, P]
    th = oracle.kernel_phase(w, basis, geom, idx)
    for K in (1, 4, 7):
        wK, bK, _ = oracle.principal_modes(w, basis, K)
        dth = np.abs(oracle.kernel_phase(wK, bK, geom, idx) - th)
        dw = w[:, 2:] - w[:, 2:] @ bK.V @ bK.V.T           # [N, 8]
        bound = np.linalg.norm(dw, axis=1)[:, None] * np.linalg.norm(ZR, axis=0)[None, :]
        assert np.all(dth <= bound * (1 + 1e-9) + 1e-12)
        assert np.max(dth) > 0.0


def test_rank_one_direction():
    rng = np.random.default_rng(5)
    N = 12
    u = rng.normal(size=N)
    v = rng.normal(size=8)
    w = _w_with_block(rng, N, np.outer(u, v))
    basis = oracle.ZernikeBasis(MODES)
    _, bK, sigma = oracle.principal_modes(w, basis, 1)
    np.testing.assert_allclose(sigma[0], np.linalg.norm(u) * np.linalg.norm(v), rtol=1e-12)
    np.testing.assert_allclose(abs(bK.V[:, 0] @ v) / np.linalg.norm(v), 1.0, rtol=1e-12)
    geom, idx = _geom_idx(8, 8)
    xh, yh = geom.coords(idx)
    B1 = bK.evaluate(xh, yh)[2]
    ref = (v / np.linalg.norm(v)) @ basis.evaluate(xh, yh)[2:]
    assert min(np.max(np.abs(B1 - ref)), np.max(np.abs(B1 + ref))) < 1e-12


def test_rejects_bad_rank():
    w = np.zeros((4, len(MODES)))
    with pytest.raises(ValueError):
        oracle.principal_modes(w, oracle.ZernikeBasis(MODES), 9)
    with pytest.raises(ValueError):
        oracle.principal_modes(w, oracle.ZernikeBasis(MODES), -1)
