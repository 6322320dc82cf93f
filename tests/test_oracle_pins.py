"""Pins of the FP64 oracle against facts it does not compute itself.

Each test fixes one part of the oracle by a closed form, an independent
numerical route, a textbook table or brute force, so that a dropped term, a
wrong sign or index, or a transposed operand anywhere in ``oracle/`` fails at
least one test.  All run on the CPU.
"""

import json
import math
import os

import numpy as np
import pytest

import oracle
from oracle import (Geometry, ZernikeBasis, MonomialBasis, forward, adjoint,
                    kernel_phase)

GOLD = os.path.join(os.path.dirname(__file__), "golden")


# --------------------------------------------------------------------------
# Zernike basis
# --------------------------------------------------------------------------

def test_paper_index_facts():
    facts = json.load(open(os.path.join(GOLD, "paper_basis_facts.json")))
    for d, nl in facts["ansi_to_nl"].items():
        assert oracle.ansi_to_nm(int(d)) == tuple(nl)
    for j, nm in facts["noll_to_nm"].items():
        assert oracle.noll_to_nm(int(j)) == tuple(nm)
    # proportionalities stated in the paper, checked at random points
    rng = np.random.default_rng(1)
    x, y = rng.uniform(-1.5, 1.5, size=(2, 50))
    z2 = oracle.zernike_nm(1, 1, x, y)
    z1 = oracle.zernike_nm(1, -1, x, y)
    z4 = oracle.zernike_nm(2, 0, x, y)
    assert np.allclose(z2 / x, z2[0] / x[0])
    assert np.allclose(z1 / y, z1[0] / y[0])
    r2 = x ** 2 + y ** 2
    assert np.allclose(np.polyfit(r2, z4, 1), [2 * math.sqrt(3), -math.sqrt(3)])


def test_ansi_roundtrip_and_noll_map():
    for d in range(66):
        n, m = oracle.ansi_to_nm(d)
        assert abs(m) <= n and (n - m) % 2 == 0
        assert oracle.nm_to_ansi(n, m) == d
    assert [oracle.noll_to_ansi(j) for j in range(4, 12)] == [4, 3, 5, 7, 8, 6, 9, 12]
    # every (n, m) up to n = 10 appears exactly once in the Noll ordering
    seen = {oracle.noll_to_nm(j) for j in range(1, 67)}
    assert len(seen) == 66


TEXTBOOK = {  # Cartesian forms of the orthonormal Zernike polynomials
    0: lambda x, y: np.ones_like(x),
    1: lambda x, y: 2 * y,
    2: lambda x, y: 2 * x,
    3: lambda x, y: 2 * math.sqrt(6) * x * y,
    4: lambda x, y: math.sqrt(3) * (2 * (x * x + y * y) - 1),
    5: lambda x, y: math.sqrt(6) * (x * x - y * y),
    6: lambda x, y: math.sqrt(8) * (3 * x * x * y - y ** 3),
    7: lambda x, y: math.sqrt(8) * (3 * (x * x + y * y) - 2) * y,
    8: lambda x, y: math.sqrt(8) * (3 * (x * x + y * y) - 2) * x,
    9: lambda x, y: math.sqrt(8) * (x ** 3 - 3 * x * y * y),
    10: lambda x, y: math.sqrt(10) * (4 * x ** 3 * y - 4 * x * y ** 3),
    11: lambda x, y: math.sqrt(10) * (4 * (x * x + y * y) - 3) * 2 * x * y,
    12: lambda x, y: math.sqrt(5) * (6 * (x * x + y * y) ** 2 - 6 * (x * x + y * y) + 1),
    13: lambda x, y: math.sqrt(10) * (4 * (x * x + y * y) - 3) * (x * x - y * y),
    14: lambda x, y: math.sqrt(10) * (x ** 4 - 6 * x * x * y * y + y ** 4),
}


def test_zernike_textbook_cartesian():
    rng = np.random.default_rng(2)
    x, y = rng.uniform(-1.9, 1.9, size=(2, 400))
    Z = ZernikeBasis(range(15)).evaluate(x, y)
    for d, fn in TEXTBOOK.items():
        np.testing.assert_allclose(Z[d], fn(x, y), rtol=1e-12, atol=1e-12)


def test_zernike_jacobi_route():
    # R_n^m(rho) = (-1)^((n-m)/2) rho^m P_{(n-m)/2}^{(m,0)}(1 - 2 rho^2)
    from scipy.special import eval_jacobi
    rng = np.random.default_rng(3)
    rho = rng.uniform(0, 1.8, 200)
    ang = rng.uniform(-np.pi, np.pi, 200)
    x, y = rho * np.cos(ang), rho * np.sin(ang)
    for d in range(45):
        n, m = oracle.ansi_to_nm(d)
        am = abs(m)
        k = (n - am) // 2
        R = (-1) ** k * rho ** am * eval_jacobi(k, am, 0, 1 - 2 * rho ** 2)
        N = math.sqrt(2 * (n + 1) / (2 if m == 0 else 1))
        ref = N * R * (np.cos(m * ang) if m >= 0 else np.sin(am * ang))
        np.testing.assert_allclose(oracle.zernike_nm(n, m, x, y), ref,
                                   rtol=1e-10, atol=1e-10)


def test_zernike_orthonormal_quadrature():
    # Gauss-Legendre in rho (weight rho) x uniform angle: exact for these
    nr, na = 24, 64
    t, wt = np.polynomial.legendre.leggauss(nr)
    rho = 0.5 * (t + 1)
    wr = 0.5 * wt * rho
    ang = 2 * np.pi * np.arange(na) / na
    R, A = np.meshgrid(rho, ang, indexing="ij")
    Wq = (wr[:, None] * np.ones(na)[None, :]) * (2 * np.pi / na) / np.pi
    Z = ZernikeBasis(range(28)).evaluate(R * np.cos(A), R * np.sin(A))
    G = np.einsum("iab,jab,ab->ij", Z, Z, Wq)
    np.testing.assert_allclose(G, np.eye(28), atol=1e-12)


def test_monomial_basis_matches_direct():
    b = MonomialBasis([(2, 0), (0, 2), (1, 1)], [[1, 0, 0], [0, 1, 0], [0.5, 0.5, 2]])
    x = np.array([0.3, -1.2]); y = np.array([2.0, 0.1])
    Z = b.evaluate(x, y)
    np.testing.assert_allclose(Z[0], x * x)
    np.testing.assert_allclose(Z[2], 0.5 * x * x + 0.5 * y * y + 2 * x * y)


# --------------------------------------------------------------------------
# Transforms
# --------------------------------------------------------------------------

def _tilt_w(u, v, geom):
    return np.stack([np.pi * np.asarray(v) * geom.R / geom.ny,
                     np.pi * np.asarray(u) * geom.R / geom.nx], axis=1)


@pytest.mark.parametrize("nx,ny", [(24, 16), (32, 32), (20, 12)])
def test_forward_integer_bins_equal_fft(nx, ny):
    rng = np.random.default_rng(10 + nx)
    geom = Geometry(nx, ny)
    u = rng.integers(-nx // 2, nx // 2, size=9)
    v = rng.integers(-ny // 2, ny // 2, size=9)
    f = rng.normal(size=(ny, nx)) + 1j * rng.normal(size=(ny, nx))
    E = forward(f, _tilt_w(u, v, geom), ZernikeBasis([1, 2]), geom)
    Ff = np.fft.fft2(f)
    ref = (-1.0) ** (u + v) * Ff[v % ny, u % nx]
    np.testing.assert_allclose(E, ref, rtol=1e-12, atol=1e-10)


def test_forward_odd_sizes_general_phase():
    nx, ny = 15, 9
    rng = np.random.default_rng(4)
    geom = Geometry(nx, ny)            # cx = 7.5, cy = 4.5
    u = rng.integers(-7, 7, size=6)
    v = rng.integers(-4, 4, size=6)
    f = rng.normal(size=(ny, nx)) + 1j * rng.normal(size=(ny, nx))
    E = forward(f, _tilt_w(u, v, geom), ZernikeBasis([1, 2]), geom)
    Ff = np.fft.fft2(f)
    ref = np.exp(2j * np.pi * (u * geom.cx / nx + v * geom.cy / ny)) * Ff[v % ny, u % nx]
    np.testing.assert_allclose(E, ref, rtol=1e-12, atol=1e-10)


def test_adjoint_integer_bins_equal_ifft():
    nx, ny = 24, 16
    rng = np.random.default_rng(5)
    geom = Geometry(nx, ny)
    # distinct bins so the sparse grid has one entry per spot
    flat = rng.choice(nx * ny, size=11, replace=False)
    v, u = np.divmod(flat, nx)
    u = u - nx // 2
    v = v - ny // 2
    y = rng.normal(size=11) + 1j * rng.normal(size=11)
    g = adjoint(y, _tilt_w(u, v, geom), ZernikeBasis([1, 2]), geom)
    grid = np.zeros((ny, nx), complex)
    grid[v % ny, u % nx] = (-1.0) ** (u + v) * y
    ref = nx * ny * np.fft.ifft2(grid)
    np.testing.assert_allclose(g, ref, rtol=1e-12, atol=1e-10)


def test_dirichlet_off_grid():
    nx, ny = 40, 28
    geom = Geometry(nx, ny)
    rng = np.random.default_rng(6)
    u = rng.uniform(-nx / 2, nx / 2, 7)
    v = rng.uniform(-ny / 2, ny / 2, 7)
    E = forward(np.ones((ny, nx)), _tilt_w(u, v, geom), ZernikeBasis([1, 2]), geom)
    ref = (np.exp(1j * np.pi * (u / nx + v / ny))
           * np.sin(np.pi * u) / np.sin(np.pi * u / nx)
           * np.sin(np.pi * v) / np.sin(np.pi * v / ny))
    np.testing.assert_allclose(E, ref, rtol=1e-11, atol=1e-10)


@pytest.mark.parametrize("n", [8, 64, 256])
def test_quadratic_gauss_sum(n):
    # basis {x^2, y^2}, origin 0, R = 1, coefficients 2 pi / n: E = -2 i n
    geom = Geometry(n, n, cx=0.0, cy=0.0, R=1.0)
    b = MonomialBasis([(2, 0), (0, 2)], [[1.0, 0.0], [0.0, 1.0]])
    w = np.array([[2 * np.pi / n, 2 * np.pi / n]])
    E = forward(np.ones((n, n)), w, b, geom)
    np.testing.assert_allclose(E, [-2j * n], rtol=1e-10, atol=1e-9 * n)


def test_conjugate_hologram_textbook_phase():
    # one spot; nearfield phase = its own kernel phase built from the
    # textbook Cartesian polynomials => E = sum A
    nx, ny = 36, 28
    geom = Geometry(nx, ny)
    rng = np.random.default_rng(7)
    modes = list(range(15))
    w = rng.normal(0, 2.0, size=(3, 15))
    jj, ii = np.mgrid[0:ny, 0:nx]
    xh = (ii - geom.cx) / geom.R
    yh = (jj - geom.cy) / geom.R
    amp = rng.uniform(0.2, 1.0, size=(ny, nx))
    for k in range(3):
        th = sum(w[k, d] * TEXTBOOK[d](xh, yh) for d in modes)
        E = forward(amp * np.exp(1j * th), w, ZernikeBasis(modes), geom)
        assert abs(E[k] - amp.sum()) < 1e-10 * amp.sum()


def test_dot_product_adjoint():
    nx, ny = 30, 22
    geom = Geometry(nx, ny)
    rng = np.random.default_rng(8)
    basis = ZernikeBasis([0, 1, 2, 3, 4, 7, 12])
    w = rng.normal(0, 3, size=(13, basis.D))
    f = rng.normal(size=(ny, nx)) + 1j * rng.normal(size=(ny, nx))
    y = rng.normal(size=13) + 1j * rng.normal(size=13)
    lhs = np.vdot(y, forward(f, w, basis, geom))        # <F f, y> as y^H F f
    rhs = np.vdot(adjoint(y, w, basis, geom), f)        # (F* y)^H f
    assert abs(lhs - rhs) < 1e-11 * abs(lhs)


def test_piston_linearity_aliasing_subsets():
    nx, ny = 26, 18
    geom = Geometry(nx, ny)
    rng = np.random.default_rng(9)
    basis = ZernikeBasis([0, 1, 2, 4, 5])
    w = rng.normal(0, 2, size=(6, 5))
    f = rng.normal(size=(ny, nx)) + 1j * rng.normal(size=(ny, nx))
    h = rng.normal(size=(ny, nx)) + 1j * rng.normal(size=(ny, nx))
    E = forward(f, w, basis, geom)
    # piston: Z_0 = 1, so +c on w[:, 0] multiplies E by exp(-i c)
    w2 = w.copy(); w2[:, 0] += 0.7
    np.testing.assert_allclose(forward(f, w2, basis, geom), E * np.exp(-0.7j), rtol=1e-12)
    # linearity
    a, b = 0.3 - 1.1j, 2.0 + 0.5j
    np.testing.assert_allclose(forward(a * f + b * h, w, basis, geom),
                               a * E + b * forward(h, w, basis, geom), rtol=1e-11, atol=1e-11)
    # aliasing: u -> u + nx is the same kernel on integer pixels (even nx)
    w3 = w.copy(); w3[:, 2] += np.pi * nx * geom.R / nx
    np.testing.assert_allclose(forward(f, w3, basis, geom), E, rtol=1e-10, atol=1e-10)
    # subsets
    sp = [4, 1]
    np.testing.assert_allclose(forward(f, w, basis, geom, spots=sp), E[sp], rtol=1e-13)
    y = rng.normal(size=6) + 1j * rng.normal(size=6)
    g = adjoint(y, w, basis, geom)
    px = np.array([0, 17, nx * ny - 1])
    np.testing.assert_allclose(adjoint(y, w, basis, geom, pixels=px),
                               g.reshape(-1)[px], rtol=1e-13)


def test_threaded_equals_serial():
    nx, ny = 64, 48
    geom = Geometry(nx, ny)
    rng = np.random.default_rng(11)
    basis = ZernikeBasis(range(10))
    w = rng.normal(0, 3, size=(40, 10))
    f = rng.normal(size=(ny, nx)) + 1j * rng.normal(size=(ny, nx))
    a = forward(f, w, basis, geom, workers=1, chunk=500)
    b = forward(f, w, basis, geom, workers=4, chunk=500)
    np.testing.assert_array_equal(a, b)


def test_bruteforce_mpmath_8x8():
    mp = pytest.importorskip("mpmath")
    mp.mp.dps = 30
    nx = ny = 8
    geom = Geometry(nx, ny)
    rng = np.random.default_rng(12)
    modes = list(range(15))
    N = 5
    w = rng.normal(0, 2.5, size=(N, 15))
    f = rng.normal(size=(ny, nx)) + 1j * rng.normal(size=(ny, nx))
    y = rng.normal(size=N) + 1j * rng.normal(size=N)

    def Z(d, x, yv):
        n, m = oracle.ansi_to_nm(d)
        am = abs(m)
        r = mp.sqrt(x * x + yv * yv)
        ang = mp.atan2(yv, x)
        k = (n - am) // 2
        R = (-1) ** k * r ** am * mp.jacobi(k, am, 0, 1 - 2 * r * r)
        N_ = mp.sqrt(mp.mpf(2 * (n + 1)) / (2 if m == 0 else 1))
        return N_ * R * (mp.cos(m * ang) if m >= 0 else mp.sin(am * ang))

    E = [mp.mpc(0)] * N
    g = np.zeros((ny, nx), complex)
    for j in range(ny):
        for i in range(nx):
            x = (mp.mpf(i) - geom.cx) / geom.R
            yv = (mp.mpf(j) - geom.cy) / geom.R
            zs = [Z(d, x, yv) for d in modes]
            acc = mp.mpc(0)
            for k in range(N):
                th = mp.fsum(mp.mpf(w[k, d]) * zs[d] for d in modes)
                E[k] += mp.expj(-th) * mp.mpc(f[j, i].real, f[j, i].imag)
                acc += mp.expj(th) * mp.mpc(y[k].real, y[k].imag)
            g[j, i] = complex(acc)
    Eo = forward(f, w, ZernikeBasis(modes), geom)
    go = adjoint(y, w, ZernikeBasis(modes), geom)
    np.testing.assert_allclose(Eo, np.array([complex(e) for e in E]), rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(go, g, rtol=1e-12, atol=1e-12)


# --------------------------------------------------------------------------
# WGS
# --------------------------------------------------------------------------

def test_one_spot_wgs_reaches_sum_amp():
    nx, ny = 32, 24
    geom = Geometry(nx, ny)
    rng = np.random.default_rng(13)
    basis = ZernikeBasis(range(10))
    w = rng.normal(0, 2, size=(1, 10))
    amp = rng.uniform(0.1, 1, size=(ny, nx))
    phi = rng.uniform(-np.pi, np.pi, size=(ny, nx))
    phi1, W1, E0, st0 = oracle.wgs_step(phi, [1.0], [1.0], amp, w, basis, geom)
    _, _, E1, st1 = oracle.wgs_step(phi1, W1, [1.0], amp, w, basis, geom)
    assert abs(abs(E1[0]) - amp.sum()) < 1e-10 * amp.sum()
    # efficiency of a single perfect spot: (sum A)^2 / (P sum A^2)
    assert abs(st1[0] - amp.sum() ** 2 / (amp.size * np.sum(amp ** 2))) < 1e-12


def _fft_wgs(phi, W, t, amp, u, v, power):
    """Independent WGS at integer bins, zero aberration, through numpy FFTs."""
    ny, nx = amp.shape
    sgn = (-1.0) ** (u + v)
    E = sgn * np.fft.fft2(amp * np.exp(1j * phi))[v % ny, u % nx]
    a = np.abs(E)
    r = (a / np.linalg.norm(a)) / (t / np.linalg.norm(t))
    W = W * r ** (-power)
    W = W / W.mean()
    grid = np.zeros((ny, nx), complex)
    grid[v % ny, u % nx] = sgn * W * t * E / a
    g = nx * ny * np.fft.ifft2(grid)
    return np.angle(g), W, E


@pytest.mark.parametrize("power", [1.0, 0.0])
def test_wgs_equals_fft_wgs_at_integer_bins(power):
    nx, ny = 32, 24
    geom = Geometry(nx, ny)
    rng = np.random.default_rng(14)
    flat = rng.choice(nx * ny, size=9, replace=False)
    v, u = np.divmod(flat, nx)
    u = u - nx // 2
    v = v - ny // 2
    w = _tilt_w(u, v, geom)
    amp = np.exp(-(((np.arange(nx) - nx / 2) / 10.0) ** 2)[None, :]
                 - (((np.arange(ny) - ny / 2) / 8.0) ** 2)[:, None])
    t = rng.uniform(0.5, 1.0, size=9)
    phi_a = rng.uniform(-np.pi, np.pi, size=(ny, nx))
    phi_b = phi_a.copy()
    Wa = np.ones(9)
    Wb = np.ones(9)
    for _ in range(6):
        phi_a, Wa, Ea, _ = oracle.wgs_step(phi_a, Wa, t, amp, w, ZernikeBasis([1, 2]), geom, power)
        phi_b, Wb, Eb = _fft_wgs(phi_b, Wb, t, amp, u, v, power)
        np.testing.assert_allclose(Ea, Eb, rtol=1e-9, atol=1e-9)
        np.testing.assert_allclose(Wa, Wb, rtol=1e-9)
        d = np.angle(np.exp(1j * (phi_a - phi_b)))
        assert np.max(np.abs(d)) < 1e-8
    if power == 0.0:
        np.testing.assert_array_equal(Wa, np.ones(9))


def test_wgs_stats_definitions():
    E = np.array([3 + 4j, 0 + 1j, 2 + 0j])
    t = np.array([1.0, 1.0, 2.0])
    amp = np.ones((2, 3))
    st = oracle.wgs_stats(E, t, amp)
    # I = |E|^2 / t^2 = [25, 1, 1]: mean 9, deviations (16, -8, -8), population
    # variance (256 + 64 + 64) / 3 = 128, so the spread is 8 sqrt(2) / 9
    assert st[0] == pytest.approx(30.0 / (6 * 6))
    assert st[1] == pytest.approx(1 - 24 / 26)
    assert st[2] == pytest.approx(8.0 * np.sqrt(2.0) / 9.0, rel=1e-15)
    assert st[3] == pytest.approx(30.0)
    # I = [1, 3]: mean 2, population std 1, spread 1/2; equal intensities
    # have spread 0 and uniformity 1
    st2 = oracle.wgs_stats(np.array([1.0 + 0j, 0 + 3j]), np.array([1.0, np.sqrt(3.0)]),
                           np.ones(4))
    assert st2[2] == pytest.approx(0.5, rel=1e-15)
    st3 = oracle.wgs_stats(np.array([2.0 + 0j, -2j, 1 + 0j]), np.array([1.0, 1.0, 0.5]),
                           np.ones(4))
    assert st3[2] == 0.0 and st3[1] == 1.0


def _bins_case(seed=17, N=9):
    nx, ny = 32, 24
    geom = Geometry(nx, ny)
    rng = np.random.default_rng(seed)
    flat = rng.choice(nx * ny, size=N, replace=False)
    v, u = np.divmod(flat, nx)
    u = u - nx // 2
    v = v - ny // 2
    amp = np.exp(-(((np.arange(nx) - nx / 2) / 10.0) ** 2)[None, :]
                 - (((np.arange(ny) - ny / 2) / 8.0) ** 2)[:, None])
    return geom, rng, u, v, _tilt_w(u, v, geom), amp


def test_feedback_with_model_amplitudes_is_the_plain_step():
    geom, rng, u, v, w, amp = _bins_case()
    t = rng.uniform(0.5, 1.0, size=len(u))
    phi = rng.uniform(-np.pi, np.pi, size=amp.shape)
    W = rng.uniform(0.5, 2.0, size=len(u))
    b = ZernikeBasis([1, 2])
    E = oracle.forward(amp * np.exp(1j * phi), w, b, geom)
    ref = oracle.wgs_step(phi, W, t, amp, w, b, geom)
    got = oracle.wgs_step(phi, W, t, amp, w, b, geom, measured=np.abs(E))
    for a, c in zip(ref, got):
        np.testing.assert_array_equal(a, c)


def test_feedback_weight_update_closed_forms():
    E = np.array([1.0 + 0j, 1j])
    # two spots, equal targets, measured 2 : 1 -> W proportional to 1/r,
    # r = (a/|a|)/(t/|t|) = (2 sqrt2/sqrt5, sqrt2/sqrt5): W = (2/3, 4/3)
    _, W = oracle.wgs_farfield(E, [1.0, 1.0], [1.0, 1.0], measured=[2.0, 1.0])
    np.testing.assert_allclose(W, [2.0 / 3.0, 4.0 / 3.0], rtol=1e-15)
    # measured proportional to the targets: the weights only renormalise
    t = np.array([0.5, 1.0, 0.8])
    E3 = np.array([1.0, 2.0, 3.0j])
    _, W3 = oracle.wgs_farfield(E3, [1.0, 2.0, 3.0], t, measured=3.0 * t)
    np.testing.assert_allclose(W3, np.array([1.0, 2.0, 3.0]) / 2.0, rtol=1e-15)
    # dark measurements keep their weight (before renormalisation)
    _, W4 = oracle.wgs_farfield(E3, [1.0, 2.0, 3.0], t, measured=[0.0, 2.0, 1.6])
    r1 = (2.0 / math.sqrt(2.0 ** 2 + 1.6 ** 2)) / (1.0 / math.sqrt(0.5 ** 2 + 1.0 + 0.8 ** 2))
    assert W4[0] / W4[1] == pytest.approx(1.0 / (2.0 / r1), rel=1e-14)


def test_phase_fixed_projection_against_fft():
    """With the farfield phases fixed, a step's new hologram is arg of the
    inverse DFT of W t exp(i psi) placed at the spot bins."""
    geom, rng, u, v, w, amp = _bins_case(seed=18)
    N = len(u)
    ny, nx = amp.shape
    t = rng.uniform(0.5, 1.0, size=N)
    phi = rng.uniform(-np.pi, np.pi, size=amp.shape)
    psi = rng.uniform(-np.pi, np.pi, size=N)
    W = rng.uniform(0.5, 2.0, size=N)
    b = ZernikeBasis([1, 2])
    phi1, W1, E, _ = oracle.wgs_step(phi, W, t, amp, w, b, geom, fixed_phase=psi)
    y, W2 = oracle.wgs_farfield(E, W, t, fixed_phase=psi)
    np.testing.assert_allclose(np.abs(y), W1 * t, rtol=1e-14)
    np.testing.assert_allclose(np.angle(y * np.exp(-1j * psi)), 0.0, atol=1e-14)
    sgn = (-1.0) ** (u + v)
    grid = np.zeros((ny, nx), complex)
    grid[v % ny, u % nx] = sgn * W1 * t * np.exp(1j * psi)
    g = nx * ny * np.fft.ifft2(grid)
    d = np.angle(np.exp(1j * (phi1 - np.angle(g))))
    assert np.max(np.abs(d)) < 1e-9


def test_phase_fixed_run_uses_the_stored_iteration():
    geom, rng, u, v, w, amp = _bins_case(seed=19)
    t = rng.uniform(0.5, 1.0, size=len(u))
    phi0 = rng.uniform(-np.pi, np.pi, size=amp.shape)
    b = ZernikeBasis([1, 2])
    phi_r, W_r, E_r, st_r, _ = oracle.wgs_run(phi0, t, amp, w, b, geom, 6,
                                              fix_phase_after=3)
    phi, W = phi0, np.ones(len(u))
    for it in range(6):
        fixed = psi if it >= 3 else None
        phi, W, E, _ = oracle.wgs_step(phi, W, t, amp, w, b, geom,
                                       fixed_phase=fixed)
        if it == 2:
            psi = np.angle(E)
    np.testing.assert_array_equal(phi, phi_r)
    np.testing.assert_array_equal(W, W_r)
    # the fixed run differs from the free one after iteration 3
    phi_f, _, _, _, _ = oracle.wgs_run(phi0, t, amp, w, b, geom, 6)
    assert np.max(np.abs(np.angle(np.exp(1j * (phi_f - phi_r))))) > 1e-6


# --------------------------------------------------------------------------
# Loss and gradient
# --------------------------------------------------------------------------

def _grad_case(nx=20, ny=14, N=7, seed=15):
    geom = Geometry(nx, ny)
    rng = np.random.default_rng(seed)
    basis = ZernikeBasis([1, 2, 3, 4, 5, 7, 12])
    w = rng.normal(0, 2, size=(N, basis.D))
    amp = rng.uniform(0.2, 1, size=(ny, nx))
    t = rng.uniform(0.5, 1, size=N)
    phi = rng.uniform(-np.pi, np.pi, size=(ny, nx))
    return geom, basis, w, amp, t, phi


def test_gradient_matches_torch_autograd_dense_kernel():
    torch = pytest.importorskip("torch")
    geom, basis, w, amp, t, phi = _grad_case()
    g, L, _ = oracle.loss_grad(phi, amp, t, w, basis, geom, lam=0.3, eps=1e-2)
    # independent route: cached dense kernel matrix + autograd (float64)
    idx = np.arange(geom.P)
    K = torch.tensor(np.exp(-1j * kernel_phase(w, basis, geom, idx)))
    ph = torch.tensor(phi, requires_grad=True)
    A = torch.tensor(amp)
    f = (A * torch.exp(1j * ph)).reshape(-1)
    E = K @ f
    s = math.sqrt(geom.P * float(np.sum(amp ** 2)) / len(t))
    Ls = torch.sum((torch.abs(E / s) ** 2 - torch.tensor(t)) ** 2)

    def wrap(d):
        return torch.remainder(d + math.pi, 2 * math.pi) - math.pi
    dx = torch.zeros_like(ph); dy = torch.zeros_like(ph)
    dx = torch.cat([wrap(ph[:, 1:] - ph[:, :-1]), torch.zeros(geom.ny, 1, dtype=ph.dtype)], 1)
    dy = torch.cat([wrap(ph[1:, :] - ph[:-1, :]), torch.zeros(1, geom.nx, dtype=ph.dtype)], 0)
    TV = torch.sum(torch.sqrt(dx ** 2 + dy ** 2 + 1e-4)) / geom.P
    Lt = Ls + 0.3 * TV
    Lt.backward()
    assert abs(L - float(Lt.detach())) < 1e-12 * abs(L)
    np.testing.assert_allclose(g, ph.grad.numpy(), rtol=1e-10, atol=1e-12)


def test_fd_update_equals_full_recompute_and_analytic():
    geom, basis, w, amp, t, phi = _grad_case(seed=16)
    lam, eps, h = 0.3, 1e-2, 1e-4
    pix = [0, 5, geom.nx + 3, geom.P - 1, geom.P // 2]
    fd = oracle.fd_grad(phi, pix, amp, t, w, basis, geom, h=h, lam=lam, eps=eps)
    full = []
    for p in pix:
        j, i = divmod(p, geom.nx)
        vals = []
        for s in (+h, -h):
            q = phi.copy(); q[j, i] += s
            vals.append(oracle.total_loss(q, amp, t, w, basis, geom, lam, eps)[0])
        full.append((vals[0] - vals[1]) / (2 * h))
    np.testing.assert_allclose(fd, full, rtol=1e-7, atol=1e-10)
    g, _, _ = oracle.loss_grad(phi, amp, t, w, basis, geom, lam=lam, eps=eps)
    ga = g.reshape(-1)[pix]
    np.testing.assert_allclose(fd, ga, rtol=1e-6, atol=1e-8 * np.max(np.abs(g)))


def test_adam_first_step_closed_form():
    # zero moments: m_hat = g and v_hat = g^2 after one update, so the phase
    # moves by lr * g / (|g| + eps)
    rng = np.random.default_rng(31)
    phi = rng.uniform(-3, 3, size=(5, 7))
    g = rng.normal(size=(5, 7)) * 10.0 ** rng.uniform(-9, 1, size=(5, 7))
    new, m, v = oracle.adam_step(phi, g, np.zeros_like(g), np.zeros_like(g), 1,
                                 lr=0.05, beta1=0.9, beta2=0.999, eps=1e-8)
    np.testing.assert_allclose(new, phi - 0.05 * g / (np.abs(g) + 1e-8),
                               rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(m, 0.1 * g, rtol=1e-15)
    np.testing.assert_allclose(v, 0.001 * g * g, rtol=1e-13)


def test_adam_matches_torch_optimizer():
    # torch.optim.Adam (float64, CPU) on a fixed sequence of gradients
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(32)
    phi = rng.uniform(-3, 3, size=40)
    grads = [rng.normal(size=40) * (1 + s) for s in range(6)]
    p = torch.tensor(phi, requires_grad=True)
    opt = torch.optim.Adam([p], lr=0.05, betas=(0.9, 0.999), eps=1e-8)
    m = np.zeros(40); v = np.zeros(40); q = phi.copy()
    for s, g in enumerate(grads, start=1):
        opt.zero_grad()
        p.grad = torch.tensor(g)
        opt.step()
        q, m, v = oracle.adam_step(q, g, m, v, s)
    np.testing.assert_allclose(q, p.detach().numpy(), rtol=1e-12, atol=1e-14)


def test_adam_run_descends_and_uses_loss_grad():
    geom, basis, w, amp, t, phi = _grad_case(seed=17)
    phi1, m, v, L = oracle.adam_run(phi, amp, t, w, basis, geom, 6, lr=0.02)
    assert L.shape == (6,) and L[-1] < L[0]
    # the first loss is the loss at the start phase
    L0, _ = oracle.total_loss(phi, amp, t, w, basis, geom)
    assert abs(L[0] - L0) <= 1e-12 * abs(L0)
    # replaying the steps by hand gives the same phase
    q = phi.copy(); mm = np.zeros_like(q); vv = np.zeros_like(q)
    for s in range(1, 7):
        g, _, _ = oracle.loss_grad(q, amp, t, w, basis, geom)
        q, mm, vv = oracle.adam_step(q, g, mm, vv, s, lr=0.02)
    np.testing.assert_allclose(phi1, q, rtol=0, atol=1e-14)


# -- gradients with respect to the kernel coefficients ----------------------
def _coef_case(seed=21, nx=14, ny=10, N=6):
    rng = np.random.default_rng(seed)
    geom = oracle.Geometry(nx, ny)
    modes = [0, 1, 2, 3, 4, 7, 12]
    basis = oracle.ZernikeBasis(modes)
    w = rng.normal(0, 0.8, size=(N, len(modes)))
    w[:, 1:3] *= 4.0
    f = rng.uniform(0.3, 1, size=(ny, nx)) * np.exp(1j * rng.uniform(-np.pi, np.pi, (ny, nx)))
    return geom, basis, w, f, rng


def test_moments_are_central_differences_of_the_fields():
    """-i M[k, d] is the derivative of E_k along w[k, d] (FP64 central
    differences, truncation ~h^2)."""
    geom, basis, w, f, _ = _coef_case()
    M = oracle.forward_moments(f, w, basis, geom)

    def central(k, d, h):
        wp = w.copy(); wp[k, d] += h
        wm = w.copy(); wm[k, d] -= h
        return (oracle.forward(f, wp, basis, geom, spots=[k])
                - oracle.forward(f, wm, basis, geom, spots=[k]))[0] / (2 * h)
    h = 1e-4
    for k in range(w.shape[0]):
        for d in range(w.shape[1]):
            # Richardson: cancels the h^2 term of the central difference
            dE = (4.0 * central(k, d, h / 2) - central(k, d, h)) / 3.0
            assert abs(dE - (-1j) * M[k, d]) < 1e-8 * max(1.0, abs(M[k, d]))


def test_piston_moment_is_the_field_and_tilt_moment_closed_form():
    """Z_0 = 1 gives M[:, 0] = E; with f = 1 and w = 0 the x-tilt moment is
    the plain sum of Z_2 = 2 xh over the grid."""
    geom, basis, w, f, _ = _coef_case()
    M = oracle.forward_moments(f, w, basis, geom)
    E = oracle.forward(f, w, basis, geom)
    np.testing.assert_allclose(M[:, 0], E, rtol=1e-13, atol=1e-12)
    # f = 1, w = 0 on the 8 x 8 SLM: M = sum_x 2 (i - nx/2) / R
    nx = ny = 8
    g = oracle.Geometry(nx, ny)
    b = oracle.ZernikeBasis([2])
    Mx = oracle.forward_moments(np.ones((ny, nx)), np.zeros((1, 1)), b, g)
    # sum_x 2 (i - nx/2)/R over the grid: ny * 2/R * sum_i (i - nx/2) = ny * 2/R * (-nx/2)
    np.testing.assert_allclose(Mx[0, 0], ny * 2.0 / g.R * (-nx / 2.0), rtol=1e-14)


def test_coef_grad_matches_torch_autograd_dense_kernel():
    torch = pytest.importorskip("torch")
    geom, basis, w, f, rng = _coef_case(seed=22)
    N = w.shape[0]
    t = rng.uniform(0.5, 1.0, N)
    s = 3.0
    E = oracle.forward(f, w, basis, geom)
    Eh = E / s
    G = 4.0 * (np.abs(Eh) ** 2 - t) * Eh / s
    g = oracle.coef_grad(f, w, basis, geom, G)
    # independent route: dense kernel built from w in torch, autograd on w
    xh, yh = geom.coords(np.arange(geom.P))
    Z = torch.tensor(basis.evaluate(xh, yh))
    wt = torch.tensor(w, requires_grad=True)
    th = wt @ Z
    Et = torch.exp(-1j * th) @ torch.tensor(f.reshape(-1))
    L = torch.sum((torch.abs(Et / s) ** 2 - torch.tensor(t)) ** 2)
    L.backward()
    np.testing.assert_allclose(g, wt.grad.numpy(), rtol=1e-10, atol=1e-12 * np.abs(g).max())


# -- in-silico spot quality --------------------------------------------------
def _dirichlet2(delta, n):
    """|sum_i exp(-2 pi i delta (i - c)/n)|^2 over n pixels (closed form)."""
    d = np.asarray(delta, dtype=np.float64)
    out = np.full(d.shape, float(n * n))
    nz = np.abs(np.sin(np.pi * d / n)) > 1e-15
    out[nz] = (np.sin(np.pi * d[nz]) / np.sin(np.pi * d[nz] / n)) ** 2
    return out


@pytest.mark.parametrize("step,win", [(1.0, 5), (0.5, 7), (0.25, 9)])
def test_window_strehl_of_a_perfect_spot_closed_form(step, win):
    """A = 1 and the hologram of one spot on an integer bin (its own tilt
    phase, written out here), no aberration: the window samples
    |D_nx(a step)|^2 |D_ny(b step)|^2 (Dirichlet kernels)."""
    nx, ny = 24, 16
    geom = Geometry(nx, ny)
    u, v = np.array([3]), np.array([-2])
    w = _tilt_w(u, v, geom)
    i = np.arange(nx)[None, :]
    j = np.arange(ny)[:, None]
    phi = 2 * np.pi * (u[0] * (i - nx / 2) / nx + v[0] * (j - ny / 2) / ny)
    S = oracle.spot_quality(np.exp(1j * phi), w, ZernikeBasis([1, 2]), geom,
                            ix=1, iy=0, win=win, step=step)
    offs = (np.arange(win) - win // 2) * step
    Ix, Iy = _dirichlet2(offs, nx), _dirichlet2(offs, ny)
    ref = Ix.max() * Iy.max() / (Ix.sum() * Iy.sum())
    assert S[0] == pytest.approx(ref, rel=1e-10)
    if step == 1.0:
        assert S[0] == pytest.approx(1.0, rel=1e-12)


def test_window_strehl_invariances_and_layout():
    nx, ny = 20, 20
    geom = Geometry(nx, ny)
    rng = np.random.default_rng(23)
    basis = ZernikeBasis([1, 2, 4, 5])
    w = rng.normal(0, 1.0, size=(3, 4))
    f = rng.uniform(0.2, 1, (ny, nx)) * np.exp(1j * rng.uniform(-np.pi, np.pi, (ny, nx)))
    S = oracle.spot_quality(f, w, basis, geom, ix=1, iy=0, win=5, step=0.5)
    S2 = oracle.spot_quality(3.7 * f, w, basis, geom, ix=1, iy=0, win=5, step=0.5)
    np.testing.assert_allclose(S, S2, rtol=1e-12)
    assert np.all((S > 0) & (S <= 1))
    S1 = oracle.spot_quality(f, w, basis, geom, ix=1, iy=0, win=1, step=0.5)
    np.testing.assert_allclose(S1, 1.0, rtol=1e-14)
    ww = oracle.window_coefficients(w, 1, 0, 0.1, 0.2, 3)
    assert ww.shape == (27, 4)
    # row (k * 3 + b) * 3 + a: x offset a - 1, y offset b - 1
    np.testing.assert_allclose(ww[(1 * 3 + 0) * 3 + 2], w[1] + [-0.2, 0.1, 0, 0], rtol=1e-15)
    np.testing.assert_allclose(ww[(2 * 3 + 1) * 3 + 1], w[2], rtol=1e-15)
