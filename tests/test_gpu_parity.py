"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Sizes here finish in seconds on the oracle while spanning several pixel
tiles (64 x 16), ragged tile and wave tails, and both directions.
"""

import math
import sys

import numpy as np
import pytest

import oracle
import workloads
from tolerance import assert_fields, assert_phase, field_errors, STEP_PHASE_MASK

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def A():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2505_08777_amd as A
    return A


def _ctx(A, nx, ny, modes, w, t=None, amp=None, **kw):
    c = A.Context(0)
    amp_t = None if amp is None else torch.tensor(amp, dtype=torch.float32, device="cuda")
    c.set_basis(nx, ny, modes=modes, amp=amp_t, **kw)
    c.set_spots(w, t)
    return c


def _cuda(x, dtype):
    return torch.tensor(np.asarray(x), dtype=dtype, device="cuda")


def _geom(c):
    return oracle.Geometry(c.nx, c.ny)


def _spots(rng, nx, ny, N, modes, sigma, R):
    """Tilts uniform over the Nyquist field, other modes ~ N(0, sigma) rad."""
    w = rng.normal(0, sigma, size=(N, len(modes)))
    if 1 in modes:
        w[:, modes.index(1)] = np.pi * rng.uniform(-ny / 2, ny / 2, N) * R / ny
    if 2 in modes:
        w[:, modes.index(2)] = np.pi * rng.uniform(-nx / 2, nx / 2, N) * R / nx
    return w


# (nx, ny, N, ANSI modes, aberration sigma in rad, pupil radius R)
CASES = [
    (256, 256, 25, [1, 2, 3, 4, 5, 6, 7, 8, 9, 12], 0.5, None),  # 4 x 16 tiles
    (100, 37, 70, [0, 1, 2, 4, 7, 12], 1.0, 50.0),               # ragged tiles, N % 64
    (64, 16, 1, [1, 2], 0.0, None),                              # one tile, one spot
    (200, 120, 130, list(range(15)), 0.8, 100.0),                # 15 modes, 3 waves
    (33, 1, 5, [2, 3, 5], 1.0, 16.5),                            # single row
    (1, 40, 3, [1, 4], 1.0, 20.0),                               # single column
    (130, 70, 200, list(range(21)), 0.5, 65.0),                  # radial order 5: 8 groups
    (512, 512, 300, [1, 2, 3, 4, 5, 6, 7, 8, 9, 12], 0.5, None), # small remainders: 2 pieces
]


@pytest.mark.parametrize("full", [False, True], ids=["auto", "full"])
@pytest.mark.parametrize("nx,ny,N,modes,sigma,R", CASES)
def test_forward_adjoint_parity(A, nx, ny, N, modes, sigma, R, full):
    _say("case", nx, ny, N, modes, sigma, R, "full" if full else "auto")
    rng = np.random.default_rng(nx * 1000 + ny)
    geom = oracle.Geometry(nx, ny, R=R)
    basis = oracle.ZernikeBasis(modes)
    w = _spots(rng, nx, ny, N, modes, sigma, geom.R)
    amp = rng.uniform(0.2, 1.0, size=(ny, nx))
    phi = rng.uniform(-np.pi, np.pi, size=(ny, nx))
    y = rng.normal(size=N) + 1j * rng.normal(size=N)
    c = A.Context(0)
    c.set_precision(full)
    c.set_basis(nx, ny, modes=modes, R=geom.R,
                amp=torch.tensor(amp, dtype=torch.float32, device="cuda"))
    c.set_spots(w)
    info = c.info()
    _say("  info", info)
    if full:
        assert info["pieces"] == 3
    else:
        assert info["pieces"] == (2 if info["rm_bound"] <= 0.5 else 3)
    assert info["range_reduce"] == (1 if info["theta_bound"] > 64 else 0)
    amp32 = amp.astype(np.float32).astype(np.float64)
    phi32 = phi.astype(np.float32).astype(np.float64)
    E = c.forward(phase=_cuda(phi32, torch.float32)).cpu().numpy()
    Eref = oracle.forward(amp32 * np.exp(1j * phi32), w, basis, geom)
    _say("  forward", field_errors(E, Eref))
    assert_fields(E, Eref, what="forward")
    y32 = y.astype(np.complex64)
    g, ph = c.adjoint(_cuda(y32, torch.complex64), field=True, phase=True)
    gref = oracle.adjoint(y32.astype(np.complex128), w, basis, geom)
    _say("  adjoint", field_errors(g.cpu().numpy(), gref))
    assert_fields(g.cpu().numpy(), gref, what="adjoint")
    assert_phase(ph.cpu().numpy(), np.angle(gref), gref, what="adjoint phase")
    # complex-field input gives the same forward as phase input
    f = _cuda((amp32 * np.exp(1j * phi32)).astype(np.complex64), torch.complex64)
    E2 = c.forward(field=f).cpu().numpy()
    assert_fields(E2, Eref, what="forward(field)")
    c.close()


def test_large_phases_take_range_reduction(A):
    # tilts far beyond the Nyquist field (aliased but a well-defined sum):
    # phase slopes of several turns per pixel push the phase bound past the
    # hardware sine's unreduced domain, so the kernels reduce explicitly
    nx, ny, N, modes = 96, 80, 45, [1, 2, 4, 7]
    rng = np.random.default_rng(96)
    geom = oracle.Geometry(nx, ny)
    basis = oracle.ZernikeBasis(modes)
    w = _spots(rng, nx, ny, N, modes, 0.7, geom.R)
    w[:, :2] *= 9.0
    amp = rng.uniform(0.2, 1.0, size=(ny, nx))
    phi = rng.uniform(-np.pi, np.pi, size=(ny, nx)).astype(np.float32)
    c = _ctx(A, nx, ny, modes, w, amp=amp)
    info = c.info()
    _say("  info", info)
    assert info["range_reduce"] == 1 and info["theta_bound"] > 64
    amp32 = amp.astype(np.float32).astype(np.float64)
    E = c.forward(phase=_cuda(phi, torch.float32)).cpu().numpy()
    Eref = oracle.forward(amp32 * np.exp(1j * phi.astype(np.float64)), w, basis, geom)
    _say("  forward", field_errors(E, Eref))
    assert_fields(E, Eref, what="forward")
    y = (rng.normal(size=N) + 1j * rng.normal(size=N)).astype(np.complex64)
    g = c.adjoint(_cuda(y, torch.complex64)).cpu().numpy()
    gref = oracle.adjoint(y.astype(np.complex128), w, basis, geom)
    _say("  adjoint", field_errors(g, gref))
    assert_fields(g, gref, what="adjoint")
    c.close()


def test_fft_bins_closed_form(A):
    nx, ny = 192, 96
    rng = np.random.default_rng(7)
    flat = rng.choice(nx * ny, size=40, replace=False)
    v, u = np.divmod(flat, nx)
    u, v = u - nx // 2, v - ny // 2
    R = min(nx, ny) / 2
    w = np.stack([np.pi * v * R / ny, np.pi * u * R / nx], 1)
    f = (rng.normal(size=(ny, nx)) + 1j * rng.normal(size=(ny, nx))).astype(np.complex64)
    c = _ctx(A, nx, ny, [1, 2], w)
    E = c.forward(field=_cuda(f, torch.complex64)).cpu().numpy()
    ref = (-1.0) ** (u + v) * np.fft.fft2(f.astype(np.complex128))[v % ny, u % nx]
    assert_fields(E, ref, what="fft bins")
    c.close()


@pytest.mark.parametrize("n", [256, 1024])
def test_quadratic_gauss_sum(A, n):
    # basis {x^2, y^2} about the origin, R = 1: E = -2 i n exactly
    c = A.Context(0)
    c.set_basis(n, n, mono_pow=[[2, 0], [0, 2]], mono_coef=[[1.0, 0.0], [0.0, 1.0]],
                cx=0.0, cy=0.0, R=1.0)
    c.set_spots(np.array([[2 * np.pi / n, 2 * np.pi / n]]))
    E = c.forward(phase=torch.zeros((n, n), dtype=torch.float32, device="cuda")).cpu().numpy()
    _say("gauss", n, E, abs(E[0] + 2j * n) / (2 * n))
    assert abs(E[0] - (-2j * n)) <= 1e-4 * 2 * n
    c.close()


def test_conjugate_hologram_and_dot_product(A):
    nx, ny = 320, 160
    rng = np.random.default_rng(8)
    modes = list(range(15))
    N = 90
    w = rng.normal(0, 3.0, size=(N, 15))
    amp = rng.uniform(0.1, 1, size=(ny, nx))
    c = _ctx(A, nx, ny, modes, w, amp=amp)
    geom = oracle.Geometry(nx, ny)
    th = oracle.kernel_phase(w[:1], oracle.ZernikeBasis(modes), geom, np.arange(nx * ny))[0]
    E = c.forward(phase=_cuda(np.angle(np.exp(1j * th)).reshape(ny, nx), torch.float32)).cpu().numpy()
    s = amp.astype(np.float32).astype(np.float64).sum()
    assert abs(E[0] - s) <= 1e-4 * s
    # <F f, y> = <f, F* y> on the GPU alone
    f = (rng.normal(size=(ny, nx)) + 1j * rng.normal(size=(ny, nx))).astype(np.complex64)
    y = (rng.normal(size=N) + 1j * rng.normal(size=N)).astype(np.complex64)
    Ff = c.forward(field=_cuda(f, torch.complex64)).cpu().numpy().astype(np.complex128)
    Fy = c.adjoint(_cuda(y, torch.complex64)).cpu().numpy().astype(np.complex128)
    lhs = np.vdot(y.astype(np.complex128), Ff)
    rhs = np.vdot(Fy, f.astype(np.complex128))
    assert abs(lhs - rhs) <= 1e-4 * np.linalg.norm(Ff) * np.linalg.norm(y)
    c.close()


def test_deterministic_bitwise(A):
    d = workloads.plain256()
    c = _ctx(A, d["nx"], d["ny"], d["modes"], d["w"], amp=d["amp"])
    ph = _cuda(d["phi0"], torch.float32)
    e1 = c.forward(phase=ph).cpu().numpy()
    e2 = c.forward(phase=ph).cpu().numpy()
    assert np.array_equal(e1.view(np.uint32), e2.view(np.uint32))
    y = _cuda(e1 / np.abs(e1), torch.complex64)
    g1 = c.adjoint(y).cpu().numpy()
    g2 = c.adjoint(y).cpu().numpy()
    assert np.array_equal(g1.view(np.uint32), g2.view(np.uint32))
    c.close()


def test_wgs_plain256_one_step_parity(A):
    """One GPU WGS step from the oracle's state at iterations 0, 1, 10, 19."""
    d = workloads.plain256()
    geom = oracle.Geometry(d["nx"], d["ny"])
    basis = oracle.ZernikeBasis(d["modes"])
    amp32 = d["amp"].astype(np.float32).astype(np.float64)
    phi0 = d["phi0"].astype(np.float32).astype(np.float64)
    keep = (0, 1, 10, 19)
    _, _, _, stats_ref, kept = oracle.wgs_run(phi0, d["t"], amp32, d["w"], basis, geom,
                                              d["n_iter"], keep=keep)
    c = _ctx(A, d["nx"], d["ny"], d["modes"], d["w"], t=d["t"], amp=d["amp"])
    for it in keep:
        phi_it, W_it = kept[it]
        phi_it32 = phi_it.astype(np.float32).astype(np.float64)
        W32 = W_it.astype(np.float32).astype(np.float64)
        ref_phi, ref_W, ref_E, ref_st = oracle.wgs_step(phi_it32, W32, d["t"], amp32,
                                                        d["w"], basis, geom)
        ph = _cuda(phi_it32, torch.float32)
        Wt = _cuda(W32, torch.float32)
        _, Wg, Eg, st = c.wgs(ph, 1, weights=Wt)
        _say("iter", it, field_errors(Eg.cpu().numpy(), ref_E))
        np.testing.assert_allclose(Wg.cpu().numpy(), ref_W, rtol=2e-4)
        # reference nearfield of the projection, for the conditioning mask
        y = ref_W * d["t"] * ref_E / np.abs(ref_E)
        gref = oracle.adjoint(y, d["w"], basis, geom)
        _say("   phase", assert_phase(ph.cpu().numpy(), ref_phi, gref,
                                  mask=STEP_PHASE_MASK, what="wgs phase @%d" % it))
        np.testing.assert_allclose(st.cpu().numpy()[0], ref_st, rtol=1e-3, atol=1e-3)
    c.close()


def test_wgs_full_run_figures(A):
    """20 iterations on the GPU: end-of-run efficiency and uniformity track
    the oracle's trajectory within 1e-3 absolute (trajectories themselves
    drift apart in FP32 vs FP64, so only the figures are compared)."""
    d = workloads.plain256()
    geom = oracle.Geometry(d["nx"], d["ny"])
    basis = oracle.ZernikeBasis(d["modes"])
    amp32 = d["amp"].astype(np.float32).astype(np.float64)
    phi0 = d["phi0"].astype(np.float32).astype(np.float64)
    _, _, _, stats_ref, _ = oracle.wgs_run(phi0, d["t"], amp32, d["w"], basis, geom, d["n_iter"])
    c = _ctx(A, d["nx"], d["ny"], d["modes"], d["w"], t=d["t"], amp=d["amp"])
    _, _, _, st = c.wgs(_cuda(phi0, torch.float32), d["n_iter"])
    st = st.cpu().numpy()
    _say("eta", st[-1, 0], stats_ref[-1, 0], "unif", st[-1, 1], stats_ref[-1, 1])
    assert abs(st[-1, 0] - stats_ref[-1, 0]) < 1e-3
    assert abs(st[-1, 1] - stats_ref[-1, 1]) < 1e-3
    c.close()


@pytest.mark.parametrize("full", [False, True], ids=["auto", "full"])
def test_largest_basis(A, full):
    """The largest supported basis: 31 modes (ANSI 0-30, radial order 7),
    28 of them non-linear, the longest record (12 matrix-core groups with 3
    pieces)."""
    nx, ny, N, modes = 128, 96, 40, list(range(31))
    rng = np.random.default_rng(31)
    geom = oracle.Geometry(nx, ny)
    basis = oracle.ZernikeBasis(modes)
    w = _spots(rng, nx, ny, N, modes, 0.05, geom.R)
    amp = rng.uniform(0.2, 1.0, size=(ny, nx)).astype(np.float32).astype(np.float64)
    phi = rng.uniform(-np.pi, np.pi, size=(ny, nx)).astype(np.float32).astype(np.float64)
    c = A.Context(0)
    c.set_precision(full)
    c.set_basis(nx, ny, modes=modes,
                amp=torch.tensor(amp, dtype=torch.float32, device="cuda"))
    c.set_spots(w)
    info = c.info()
    _say("  info", info)
    assert info["nonlinear"] == 28
    if full:
        assert info["groups"] == 12
    E = c.forward(phase=_cuda(phi, torch.float32)).cpu().numpy()
    Eref = oracle.forward(amp * np.exp(1j * phi), w, basis, geom)
    _say("  forward", field_errors(E, Eref))
    assert_fields(E, Eref, what="forward, 31 modes")
    y = (rng.normal(size=N) + 1j * rng.normal(size=N)).astype(np.complex64)
    g = c.adjoint(_cuda(y, torch.complex64)).cpu().numpy()
    gref = oracle.adjoint(y.astype(np.complex128), w, basis, geom)
    _say("  adjoint", field_errors(g, gref))
    assert_fields(g, gref, what="adjoint, 31 modes")
    M = c.forward_moments(_cuda(phi, torch.float32)).cpu().numpy()
    Mref = oracle.forward_moments(amp * np.exp(1j * phi), w, basis, geom)
    for d in range(len(modes)):
        assert_fields(M[:, d], Mref[:, d], what="moments, mode %d" % d)
    c.close()


def test_many_spots_small_slm(A):
    """100 000 spots on a 64 x 48 SLM (more spots than pixels): sampled
    spots of the forward and all pixels of the adjoint."""
    nx, ny, N, modes = 64, 48, 100000, [1, 2, 3, 4, 5, 7]
    rng = np.random.default_rng(100)
    geom = oracle.Geometry(nx, ny)
    basis = oracle.ZernikeBasis(modes)
    w = _spots(rng, nx, ny, N, modes, 0.5, geom.R)
    amp = rng.uniform(0.2, 1.0, size=(ny, nx)).astype(np.float32).astype(np.float64)
    phi = rng.uniform(-np.pi, np.pi, size=(ny, nx)).astype(np.float32).astype(np.float64)
    c = _ctx(A, nx, ny, modes, w, amp=amp)
    E = c.forward(phase=_cuda(phi, torch.float32)).cpu().numpy()
    sel = np.sort(rng.choice(N, size=512, replace=False))
    Eref = oracle.forward(amp * np.exp(1j * phi), w, basis, geom, spots=sel)
    _say("  forward", field_errors(E[sel], Eref))
    assert_fields(E[sel], Eref, what="forward, 1e5 spots")
    y = (rng.normal(size=N) + 1j * rng.normal(size=N)).astype(np.complex64)
    g = c.adjoint(_cuda(y, torch.complex64)).cpu().numpy()
    gref = oracle.adjoint(y.astype(np.complex128), w, basis, geom)
    _say("  adjoint", field_errors(g, gref))
    assert_fields(g, gref, what="adjoint, 1e5 spots")
    c.close()


def test_maximum_spot_count(A):
    """The largest supported spot count (2^20) on one 64 x 16 tile: sampled
    spots of the forward, sampled pixels of the adjoint (each a sum over
    all 2^20 spots), and one spot more is refused with the context kept."""
    from paper_2505_08777_amd import _lib
    nx, ny, modes = 64, 16, [1, 2, 4]
    N = _lib.MAX_SPOTS
    rng = np.random.default_rng(2020)
    geom = oracle.Geometry(nx, ny)
    basis = oracle.ZernikeBasis(modes)
    w = _spots(rng, nx, ny, N, modes, 0.7, geom.R)
    amp = rng.uniform(0.2, 1.0, size=(ny, nx)).astype(np.float32).astype(np.float64)
    phi = rng.uniform(-np.pi, np.pi, size=(ny, nx)).astype(np.float32).astype(np.float64)
    c = _ctx(A, nx, ny, modes, w, amp=amp)
    E = c.forward(phase=_cuda(phi, torch.float32)).cpu().numpy()
    sel = np.sort(np.concatenate([[0, N - 1], rng.choice(N, size=510, replace=False)]))
    Eref = oracle.forward(amp * np.exp(1j * phi), w, basis, geom, spots=sel)
    _say("  forward", field_errors(E[sel], Eref))
    assert_fields(E[sel], Eref, what="forward, 2^20 spots")
    y = (rng.normal(size=N) + 1j * rng.normal(size=N)).astype(np.complex64)
    g = c.adjoint(_cuda(y, torch.complex64)).cpu().numpy().reshape(-1)
    pix = np.sort(rng.choice(nx * ny, size=48, replace=False))
    gref = oracle.adjoint(y.astype(np.complex128), w, basis, geom, pixels=pix)
    _say("  adjoint", field_errors(g[pix], gref))
    assert_fields(g[pix], gref, what="adjoint, 2^20 spots")
    w_more = np.zeros((N + 1, len(modes)))
    assert _lib.lib.ash_set_spots(c._h, N + 1, w_more.ctypes.data,
                                  None) == _lib.EUNSUPPORTED
    E2 = c.forward(phase=_cuda(phi, torch.float32)).cpu().numpy()
    assert np.array_equal(E, E2)
    c.close()


@pytest.mark.parametrize("nx,ny", [(65536, 16), (16, 65536)])
def test_maximum_side(A, nx, ny):
    """The largest supported side (65536 pixels): every pixel of both
    transforms for a few spots, and one pixel more is refused."""
    from paper_2505_08777_amd import _lib
    assert max(nx, ny) == _lib.MAX_SIDE
    modes, N = [1, 2, 4, 5], 6
    rng = np.random.default_rng(nx + 3 * ny)
    geom = oracle.Geometry(nx, ny, R=max(nx, ny) / 2.0)  # pupil along the strip
    basis = oracle.ZernikeBasis(modes)
    w = _spots(rng, nx, ny, N, modes, 0.5, geom.R)
    amp = rng.uniform(0.2, 1.0, size=(ny, nx)).astype(np.float32).astype(np.float64)
    phi = rng.uniform(-np.pi, np.pi, size=(ny, nx)).astype(np.float32).astype(np.float64)
    c = _ctx(A, nx, ny, modes, w, amp=amp, R=geom.R)
    E = c.forward(phase=_cuda(phi, torch.float32)).cpu().numpy()
    Eref = oracle.forward(amp * np.exp(1j * phi), w, basis, geom)
    _say("  forward", field_errors(E, Eref))
    assert_fields(E, Eref, what="forward, side %d" % max(nx, ny))
    y = (rng.normal(size=N) + 1j * rng.normal(size=N)).astype(np.complex64)
    g = c.adjoint(_cuda(y, torch.complex64)).cpu().numpy()
    gref = oracle.adjoint(y.astype(np.complex128), w, basis, geom)
    _say("  adjoint", field_errors(g, gref))
    assert_fields(g, gref, what="adjoint, side %d" % max(nx, ny))
    c.close()
    c = A.Context(0)
    pw, cf = A.zernike_table(modes)
    pw = np.ascontiguousarray(pw, np.int32)
    cf = np.ascontiguousarray(cf, np.float64)
    bx, by = (nx + 1, ny) if nx > ny else (nx, ny + 1)
    assert _lib.lib.ash_set_basis(c._h, bx, by, bx / 2.0, by / 2.0, 8.0,
                                  len(modes), pw.shape[0], pw.ctypes.data,
                                  cf.ctypes.data, None) == _lib.EUNSUPPORTED
    c.close()


def _disk_peak_valley(d, n=801):
    """Peak-to-valley of the orthonormal Zernike with ANSI index d over the
    unit disk (dense grid)."""
    x, y = np.meshgrid(np.linspace(-1, 1, n), np.linspace(-1, 1, n))
    inside = x ** 2 + y ** 2 <= 1.0
    z = oracle.zernike_nm(*oracle.ansi_to_nm(d), x[inside], y[inside])
    return float(z.max() - z.min())


def test_paper_magnitudes_pyramid_and_astigmatism(A):
    """Inputs at the magnitudes the paper reports: a Zernike pyramid (one
    spot per mode of radial orders 2-4, each carrying +-5 rad peak-valley of
    its own mode over the pupil, "Aberration-Space Holography"), and a field
    of spots whose astigmatism Z_5 reaches -30 rad (Fig. 4's principal-mode
    discussion) on top of unit-size other aberrations."""
    # pyramid: 12 spots, basis = tilts + ANSI 3..14
    nx = ny = 384
    pyr = list(range(3, 15))
    modes = [1, 2] + pyr
    geom = oracle.Geometry(nx, ny)
    basis = oracle.ZernikeBasis(modes)
    w = np.zeros((len(pyr), len(modes)))
    k = 0
    for n_rad, first in ((2, 3), (3, 6), (4, 10)):
        for col in range(n_rad + 1):
            u = 24.0 * (col - n_rad / 2.0)
            v = 24.0 * (n_rad - 3)
            w[k, 0] = np.pi * v * geom.R / ny
            w[k, 1] = np.pi * u * geom.R / nx
            w[k, 2 + k] = 10.0 / _disk_peak_valley(first + col)
            k += 1
    rng = np.random.default_rng(141)
    amp = rng.uniform(0.2, 1.0, size=(ny, nx)).astype(np.float32).astype(np.float64)
    phi = rng.uniform(-np.pi, np.pi, size=(ny, nx)).astype(np.float32).astype(np.float64)
    c = _ctx(A, nx, ny, modes, w, amp=amp)
    E = c.forward(phase=_cuda(phi, torch.float32)).cpu().numpy()
    Eref = oracle.forward(amp * np.exp(1j * phi), w, basis, geom)
    _say("  pyramid forward", field_errors(E, Eref))
    assert_fields(E, Eref, what="pyramid forward")
    y = (rng.normal(size=len(pyr)) + 1j * rng.normal(size=len(pyr))).astype(np.complex64)
    g = c.adjoint(_cuda(y, torch.complex64)).cpu().numpy()
    gref = oracle.adjoint(y.astype(np.complex128), w, basis, geom)
    _say("  pyramid adjoint", field_errors(g, gref))
    assert_fields(g, gref, what="pyramid adjoint")
    c.close()
    # astigmatism down to -30 rad over the field, 10-mode basis
    nx = ny = 512
    N = 300
    modes = [1, 2, 3, 4, 5, 6, 7, 8, 9, 12]
    geom = oracle.Geometry(nx, ny)
    basis = oracle.ZernikeBasis(modes)
    rng = np.random.default_rng(341)
    w = _spots(rng, nx, ny, N, modes, 1.0, geom.R)
    w[:, modes.index(5)] = rng.uniform(-30.0, -20.0, N)
    amp = rng.uniform(0.2, 1.0, size=(ny, nx)).astype(np.float32).astype(np.float64)
    phi = rng.uniform(-np.pi, np.pi, size=(ny, nx)).astype(np.float32).astype(np.float64)
    c = _ctx(A, nx, ny, modes, w, amp=amp)
    _say("  info", c.info())
    E = c.forward(phase=_cuda(phi, torch.float32)).cpu().numpy()
    Eref = oracle.forward(amp * np.exp(1j * phi), w, basis, geom)
    _say("  astigmatism forward", field_errors(E, Eref))
    assert_fields(E, Eref, what="astigmatism forward")
    y = (rng.normal(size=N) + 1j * rng.normal(size=N)).astype(np.complex64)
    g = c.adjoint(_cuda(y, torch.complex64)).cpu().numpy()
    gref = oracle.adjoint(y.astype(np.complex128), w, basis, geom)
    _say("  astigmatism adjoint", field_errors(g, gref))
    assert_fields(g, gref, what="astigmatism adjoint")
    c.close()


def test_phase_bound_guard(A):
    """A high-order basis on a small pupil (ANSI 0-27, radial order 6, on
    R = 38 pixels of a 128 x 96 SLM, corners at rho ~ 2.1): scaled so the
    in-tile phase bound is about 140 turns the transforms still meet the
    field bar in both precisions; scaled to about 530 turns (kernels
    changing by several turns between neighbouring pixels) set_spots is
    refused and the context holds no spots."""
    from paper_2505_08777_amd import _lib
    nx, ny, R, N = 128, 96, 38.0, 60
    modes = list(range(28))
    rng = np.random.default_rng(6)
    geom = oracle.Geometry(nx, ny, R=R)
    basis = oracle.ZernikeBasis(modes)
    w0 = rng.normal(0, 1.0, size=(N, len(modes)))
    w0[:, 1] = np.pi * rng.uniform(-ny / 2, ny / 2, N) * R / ny
    w0[:, 2] = np.pi * rng.uniform(-nx / 2, nx / 2, N) * R / nx
    nl = [k for k in modes if k not in (0, 1, 2)]
    amp = rng.uniform(0.2, 1.0, size=(ny, nx)).astype(np.float32).astype(np.float64)
    phi = rng.uniform(-np.pi, np.pi, size=(ny, nx)).astype(np.float32).astype(np.float64)
    y = (rng.normal(size=N) + 1j * rng.normal(size=N)).astype(np.complex64)
    c = A.Context(0)
    c.set_basis(nx, ny, modes=modes, R=R,
                amp=torch.tensor(amp, dtype=torch.float32, device="cuda"))
    # the remainder bound is linear in the non-linear coefficients
    w = w0.copy()
    w[:, nl] *= 1e-3
    c.set_spots(w)
    rm1 = c.info()["rm_bound"]
    for full in (False, True):
        w = w0.copy()
        w[:, nl] *= 1e-3 * 80.0 / rm1
        c.set_precision(full)
        c.set_spots(w)
        info = c.info()
        _say("  accepted", "full" if full else "auto", info)
        assert 64 < info["theta_bound"] <= 256 and info["range_reduce"] == 1
        E = c.forward(phase=_cuda(phi, torch.float32)).cpu().numpy()
        Eref = oracle.forward(amp * np.exp(1j * phi), w, basis, geom)
        g = c.adjoint(_cuda(y, torch.complex64)).cpu().numpy()
        gref = oracle.adjoint(y.astype(np.complex128), w, basis, geom)
        _say("    forward", field_errors(E, Eref), "adjoint", field_errors(g, gref))
        assert_fields(E, Eref, what="forward below the phase bound")
        assert_fields(g, gref, what="adjoint below the phase bound")
    w = w0.copy()
    w[:, nl] *= 1e-3 * 320.0 / rm1
    with pytest.raises(A.AshError) as exc:
        c.set_spots(w)
    _say("  refused:", exc.value, c.info())
    assert exc.value.code == _lib.EUNSUPPORTED
    assert c.info()["theta_bound"] > 256
    with pytest.raises(A.AshError) as exc:
        c.forward(phase=_cuda(phi, torch.float32))
    assert exc.value.code == _lib.ENOTREADY
    c.close()
