"""Host-side checks of the C ABI: the library loads, exports every symbol
that include/ash.h declares, expands Zernike polynomials exactly and
rejects bad arguments with the documented codes.  No GPU compute."""

import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ash.h")

A = pytest.importorskip("paper_2505_08777_amd")
from paper_2505_08777_amd import _lib  # noqa: E402
import oracle  # noqa: E402


def declared_symbols(header=HEADER):
    src = open(header).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ash_[a-z_0-9]+)\s*\(", src)))


# each header of include/ and the library that implements it
LIBS = {"ash.h": "libash.so", "ash_ubench.h": "libash_ubench.so"}


def test_exports_every_declared_symbol():
    syms = declared_symbols()
    assert "ash_forward" in syms and "ash_wgs_iterate" in syms
    headers = sorted(f for f in os.listdir(os.path.join(ROOT, "include"))
                     if f.endswith(".h"))
    assert headers == sorted(LIBS)
    for h in headers:
        lib = ctypes.CDLL(os.path.join(os.path.dirname(_lib.LIB_PATH), LIBS[h]))
        syms = declared_symbols(os.path.join(ROOT, "include", h))
        assert syms
        missing = [s for s in syms if not hasattr(lib, s)]
        assert not missing, (h, missing)


def test_status_codes_match_header():
    src = open(HEADER).read()
    codes = dict((m.group(1), int(m.group(2))) for m in
                 re.finditer(r"#define (ASH_E[A-Z]+) \((-\d+)\)", src))
    assert codes == {"ASH_EINVAL": _lib.EINVAL, "ASH_ESHAPE": _lib.ESHAPE,
                     "ASH_ENOTREADY": _lib.ENOTREADY,
                     "ASH_EUNSUPPORTED": _lib.EUNSUPPORTED,
                     "ASH_ENOMEM": _lib.ENOMEM, "ASH_EHIP": _lib.EHIP}
    for c in list(codes.values()) + [0]:
        assert _lib.strerror(c) != "unknown error"
    assert _lib.strerror(-99) == "unknown error"


def test_limits_match_header():
    src = open(HEADER).read()
    lim = dict((m.group(1), int(m.group(2))) for m in
               re.finditer(r"#define ASH_MAX_([A-Z_]+) (\d+)", src))
    assert lim == {"MODES": _lib.MAX_MODES, "NONLINEAR": _lib.MAX_NONLINEAR,
                   "MONOMIALS": _lib.MAX_MONOMIALS,
                   "DEGREE": _lib.MAX_DEGREE, "SIDE": _lib.MAX_SIDE,
                   "SPOTS": _lib.MAX_SPOTS,
                   "PRINCIPAL_MODES": _lib.MAX_PRINCIPAL_MODES}


@pytest.mark.parametrize("ansi", range(0, 66))
def test_zernike_expansion_matches_radial_formula(ansi):
    pw, cf = A.zernike_monomials(ansi)
    rng = np.random.default_rng(ansi)
    x, y = rng.uniform(-1.9, 1.9, size=(2, 64))
    val = sum(c * x ** p * y ** q for (p, q), c in zip(pw, cf))
    n, m = oracle.ansi_to_nm(ansi)
    ref = oracle.zernike_nm(n, m, x, y)
    np.testing.assert_allclose(val, ref, rtol=1e-10, atol=1e-9)


def test_zernike_table_union():
    pw, cf = A.zernike_table([1, 2, 4, 12])
    assert cf.shape == (4, pw.shape[0])
    x, y = 0.3, -0.7
    mono = np.array([x ** p * y ** q for p, q in pw])
    np.testing.assert_allclose(cf @ mono, [oracle.zernike_nm(*oracle.ansi_to_nm(d), x, y)
                                           for d in [1, 2, 4, 12]], rtol=1e-12)


def test_zernike_expansion_errors():
    lib = _lib.lib
    pw = np.zeros((4, 2), np.int32)
    cf = np.zeros(4)
    assert lib.ash_zernike_monomials(-1, 4, pw.ctypes.data, cf.ctypes.data) == _lib.EINVAL
    assert lib.ash_zernike_monomials(3, 4, None, None) == _lib.EINVAL
    # Z_12 has 6 terms: a cap of 4 is too small
    assert lib.ash_zernike_monomials(12, 4, pw.ctypes.data, cf.ctypes.data) == _lib.EUNSUPPORTED
    # radial order 13 exceeds the supported degree
    assert lib.ash_zernike_monomials(13 * 15 // 2 + 1, 4, pw.ctypes.data, cf.ctypes.data) == _lib.EUNSUPPORTED


def test_null_context_and_arguments():
    lib = _lib.lib
    assert lib.ash_create(None, 0, None) == _lib.EINVAL
    assert lib.ash_destroy(None) == _lib.EINVAL
    assert lib.ash_sync(None) == _lib.EINVAL
    assert lib.ash_set_spots(None, 1, None, None) == _lib.EINVAL
    assert lib.ash_forward(None, None, None, None) == _lib.EINVAL
    assert lib.ash_adjoint(None, None, None, None) == _lib.EINVAL
    assert lib.ash_wgs_iterate(None, None, None, 1, None, None, None) == _lib.EINVAL
    assert lib.ash_last_error(None) == b"null context"  # after ash_create(NULL)
    assert lib.ash_version() >= 100


def _check_basis(nx, ny, cx, cy, R, D, pw, cf):
    lib = _lib.lib
    lib.ash_check_basis.restype = ctypes.c_int
    lib.ash_check_basis.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                    ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                    ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                    ctypes.POINTER(ctypes.c_char_p)]
    why = ctypes.c_char_p()
    n_mono = 0 if pw is None else pw.shape[0]
    rc = lib.ash_check_basis(nx, ny, cx, cy, R, D, n_mono,
                             None if pw is None else pw.ctypes.data,
                             None if cf is None else cf.ctypes.data,
                             ctypes.byref(why))
    return rc, why.value.decode()


def _check_spots(N, D, w, t):
    lib = _lib.lib
    lib.ash_check_spots.restype = ctypes.c_int
    lib.ash_check_spots.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                    ctypes.c_void_p, ctypes.POINTER(ctypes.c_char_p)]
    why = ctypes.c_char_p()
    rc = lib.ash_check_spots(N, D, None if w is None else w.ctypes.data,
                             None if t is None else t.ctypes.data,
                             ctypes.byref(why))
    return rc, why.value.decode()


def test_setup_argument_checks_without_a_device():
    """ash_check_basis / ash_check_spots (the checks ash_set_basis and
    ash_set_spots run first) return every documented code on the CPU."""
    pw, cf = zernike_table_np([1, 2, 4])
    assert _check_basis(64, 48, 32.0, 24.0, 24.0, 3, pw, cf) == (_lib.OK, "")
    bad = [
        ((0, 48, 32.0, 24.0, 24.0, 3, pw, cf), _lib.EINVAL, "out of range"),
        ((70000, 48, 32.0, 24.0, 24.0, 3, pw, cf), _lib.EUNSUPPORTED, "out of range"),
        ((64, 48, 32.0, 24.0, 0.0, 3, pw, cf), _lib.EINVAL, "R > 0"),
        ((64, 48, float("nan"), 24.0, 24.0, 3, pw, cf), _lib.EINVAL, "finite"),
        ((64, 48, 32.0, 24.0, 24.0, 3, None, cf), _lib.EINVAL, "non-null"),
        ((64, 48, 32.0, 24.0, 24.0, 0, pw, cf), _lib.EINVAL, "D, n_mono"),
        ((64, 48, 32.0, 24.0, 24.0, 40, pw, np.zeros((40, pw.shape[0]))),
         _lib.EUNSUPPORTED, "too many"),
    ]
    neg = pw.copy()
    neg[1, 0] = -1
    bad.append(((64, 48, 32.0, 24.0, 24.0, 3, neg, cf), _lib.EINVAL, "negative"))
    rep = pw.copy()
    rep[1] = rep[0]
    bad.append(((64, 48, 32.0, 24.0, 24.0, 3, rep, cf), _lib.EINVAL, "repeated"))
    high = np.array([[13, 0]], np.int32)
    bad.append(((64, 48, 32.0, 24.0, 24.0, 1, high, np.ones((1, 1))),
                _lib.EUNSUPPORTED, "degree"))
    nan = cf.copy()
    nan[2, 0] = np.nan
    bad.append(((64, 48, 32.0, 24.0, 24.0, 3, pw, nan), _lib.EINVAL, "non-finite"))
    for args, code, text in bad:
        rc, why = _check_basis(*args)
        assert rc == code and text in why, (args[:6], rc, why)
    w = np.random.default_rng(1).normal(size=(5, 3))
    t = np.ones(5, np.float32)
    assert _check_spots(5, 3, w, t) == (_lib.OK, "")
    assert _check_spots(5, 3, w, None) == (_lib.OK, "")
    assert _check_spots(0, 3, w, t)[0] == _lib.EINVAL
    assert _check_spots(5, 3, None, t)[0] == _lib.EINVAL
    assert _check_spots(_lib.MAX_SPOTS + 1, 3, w, t)[0] == _lib.EUNSUPPORTED
    wn = w.copy()
    wn[4, 2] = np.inf
    assert _check_spots(5, 3, wn, t) == (_lib.EINVAL, "non-finite spot coefficient")
    for tv in (0.0, -1.0, np.nan):
        tb = t.copy()
        tb[3] = tv
        assert _check_spots(5, 3, w, tb)[0] == _lib.EINVAL


def zernike_table_np(modes):
    from paper_2505_08777_amd.basis import zernike_table
    pw, cf = zernike_table(modes)
    return np.ascontiguousarray(pw, np.int32), np.ascontiguousarray(cf, np.float64)


def test_create_without_gpu_reports_hip_error():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = ctypes.c_void_p()
    assert _lib.lib.ash_create(ctypes.byref(h), 0, None) == _lib.EHIP


# -- principal isoplanatic modes (host-only entry point) ---------------------
PM_MODES = [0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 12, 13]


def _pm_case(seed, N, rank=None):
    rng = np.random.default_rng(seed)
    nr = len(PM_MODES) - 3
    if rank is None:
        WR = rng.normal(0, 1.0, size=(N, nr)) * np.linspace(2.0, 0.1, nr)
    else:
        WR = rng.normal(size=(N, rank)) @ rng.normal(size=(rank, nr))
    w = np.concatenate([rng.normal(size=(N, 1)), rng.uniform(-40, 40, size=(N, 2)), WR], axis=1)
    return w


@pytest.mark.parametrize("N,K", [(40, 3), (7, 9), (200, 1), (5, 0), (30, 9)])
def test_principal_modes_match_oracle(N, K):
    """Singular values and the truncated kernel phases against the oracle
    (numpy's SVD); the phases do not depend on singular-vector signs."""
    w = _pm_case(N * 10 + K, N)
    pw, cf = A.zernike_table(PM_MODES)
    cfK, wK, sigma = A.principal_modes(pw, cf, w, K)
    basis = oracle.ZernikeBasis(PM_MODES)
    wr, br, sr = oracle.principal_modes(w, basis, K)
    np.testing.assert_allclose(sigma, sr, rtol=1e-10, atol=1e-12 * sr[0])
    assert cfK.shape == (3 + K, pw.shape[0]) and wK.shape == (N, 3 + K)
    geom = oracle.Geometry(40, 30)
    idx = np.arange(geom.P)
    th = oracle.kernel_phase(wK, oracle.MonomialBasis(pw, cfK), geom, idx)
    th_ref = oracle.kernel_phase(wr, br, geom, idx)
    assert np.max(np.abs(th - th_ref)) < 1e-9 * max(1.0, np.max(np.abs(th_ref)))
    # kept modes first and unchanged
    np.testing.assert_array_equal(wK[:, :3], w[:, :3])
    np.testing.assert_array_equal(cfK[:3], cf[:3])


def test_principal_modes_rank_k_exact():
    w = _pm_case(3, 60, rank=4)
    pw, cf = A.zernike_table(PM_MODES)
    cfK, wK, sigma = A.principal_modes(pw, cf, w, 4)
    assert np.all(sigma[4:] < 1e-12 * sigma[0])
    geom = oracle.Geometry(24, 24)
    idx = np.arange(geom.P)
    th = oracle.kernel_phase(w, oracle.ZernikeBasis(PM_MODES), geom, idx)
    thK = oracle.kernel_phase(wK, oracle.MonomialBasis(pw, cfK), geom, idx)
    assert np.max(np.abs(thK - th)) < 1e-10


def test_principal_modes_of_a_44_mode_calibration():
    """The paper's calibration size: 44 modes (ANSI 1-44, radial orders up
    to 8; tilts kept), rotated onto K = 8 principal modes, against the
    oracle; the output fits the transforms (2 + 8 modes)."""
    modes = list(range(1, 45))
    rng = np.random.default_rng(44)
    N, nr = 120, 42
    WR = rng.normal(size=(N, 6)) @ rng.normal(size=(6, nr)) \
        + 0.05 * rng.normal(size=(N, nr))
    w = np.concatenate([rng.uniform(-40, 40, size=(N, 2)), WR], axis=1)
    pw, cf = A.zernike_table(modes)
    assert cf.shape[0] == 44 > _lib.MAX_MODES
    cfK, wK, sigma = A.principal_modes(pw, cf, w, 8)
    assert cfK.shape[0] == 10 and wK.shape == (N, 10)
    wr, br, sr = oracle.principal_modes(w, oracle.ZernikeBasis(modes), 8)
    np.testing.assert_allclose(sigma, sr, rtol=1e-10, atol=1e-12 * sr[0])
    geom = oracle.Geometry(36, 28)
    idx = np.arange(geom.P)
    th = oracle.kernel_phase(wK, oracle.MonomialBasis(pw, cfK), geom, idx)
    th_ref = oracle.kernel_phase(wr, br, geom, idx)
    assert np.max(np.abs(th - th_ref)) < 1e-9 * max(1.0, np.max(np.abs(th_ref)))
    # one mode more than the limit is refused
    big = list(range(0, _lib.MAX_PRINCIPAL_MODES + 1))
    pwb, cfb = A.zernike_table(big)
    wb = rng.normal(size=(5, len(big)))
    with pytest.raises(A.AshError):
        A.principal_modes(pwb, cfb, wb, 1)


def test_principal_modes_errors():
    pw, cf = A.zernike_table(PM_MODES)
    w = _pm_case(1, 10)
    with pytest.raises(A.AshError):
        A.principal_modes(pw, cf, w, 10)          # only 9 modes rotate
    with pytest.raises(A.AshError):
        A.principal_modes(pw, cf, w, -1)
    w2 = w.copy()
    w2[3, 5] = np.nan
    with pytest.raises(A.AshError):
        A.principal_modes(pw, cf, w2, 2)
    assert _lib.lib.ash_principal_modes(0, 1, 1, None, None, None, 0, None,
                                        None, None, None) == _lib.EINVAL


def test_window_coefficients_match_oracle_and_errors():
    rng = np.random.default_rng(31)
    w = rng.normal(size=(4, 6))
    for nx, ny, R, step in ((64, 48, 24.0, 0.3), (1920, 1200, 600.0, -0.25)):
        geom = oracle.Geometry(nx, ny, R=R)
        a = A.window_coefficients(w, 2, 1, nx, ny, R, step, 7)
        b = oracle.window_coefficients(w, 2, 1,
                                       *oracle.window_spacing(geom, step), 7)
        np.testing.assert_allclose(a, b, rtol=0, atol=1e-14)
    out = np.zeros(4 * 49 * 6)
    L = _lib.lib

    def call(ix=2, iy=1, nx=64, ny=48, R=24.0, step=0.3, win=7):
        return L.ash_window_coefficients(4, 6, w.ctypes.data, ix, iy, nx, ny,
                                         R, step, win, out.ctypes.data)
    assert call() == _lib.OK
    assert call(win=6) == _lib.EINVAL           # even window
    assert call(iy=2) == _lib.EINVAL            # ix == iy
    assert call(ix=6) == _lib.EINVAL            # ix >= D
    assert call(step=float("nan")) == _lib.EINVAL
    assert call(R=0.0) == _lib.EINVAL
    assert call(nx=0) == _lib.EINVAL
    assert L.ash_window_strehl(None, None, 1, 1, None) == _lib.EINVAL
