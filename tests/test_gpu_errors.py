"""Argument validation through the C ABI with a live context: each bad call
returns its documented code, enqueues nothing and leaves the context as it
was (a later valid call gives bitwise the same result as before the bad
one)."""

import ctypes
import math
import sys

import numpy as np

import pytest

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


def _p(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def test_error_codes_and_unchanged_state(A):
    from paper_2505_08777_amd import _lib
    L = _lib.lib
    EINVAL, ESHAPE, ENOTREADY, EUNSUP = (_lib.EINVAL, _lib.ESHAPE,
                                        _lib.ENOTREADY, _lib.EUNSUPPORTED)
    c = A.Context(0)
    h = c._h
    nx, ny = 64, 48
    ph = torch.zeros((ny, nx), dtype=torch.float32, device="cuda")
    E = torch.empty(4, dtype=torch.complex64, device="cuda")
    w = np.random.default_rng(0).normal(size=(4, 3))
    # nothing set yet
    assert L.ash_set_spots(h, 4, w.ctypes.data, None) == ENOTREADY
    assert L.ash_forward(h, _p(ph), None, _p(E)) == ENOTREADY
    assert L.ash_forward_moments(h, _p(ph), _p(E)) == ENOTREADY
    assert L.ash_window_strehl(h, _p(ph), 1, 1, _p(E)) == ENOTREADY
    assert L.ash_last_error(h).decode() != ""
    # basis validation
    pw, cf = A.zernike_table([1, 2, 4])
    pw = np.ascontiguousarray(pw, np.int32)
    cf = np.ascontiguousarray(cf, np.float64)

    def sb(nx_, ny_, R, D, n_mono, pw_, cf_):
        return L.ash_set_basis(h, nx_, ny_, nx_ / 2.0, ny_ / 2.0, R, D, n_mono,
                               pw_.ctypes.data, cf_.ctypes.data, None)
    assert sb(0, ny, 24.0, 3, pw.shape[0], pw, cf) == EINVAL
    assert sb(nx, ny, 0.0, 3, pw.shape[0], pw, cf) == EINVAL
    assert sb(nx, ny, 24.0, 40, pw.shape[0], pw, np.zeros((40, pw.shape[0]))) == EUNSUP
    bad = cf.copy()
    bad[2, 0] = np.nan
    assert sb(nx, ny, 24.0, 3, pw.shape[0], pw, bad) == EINVAL
    rep = pw.copy()
    rep[1] = rep[0]
    assert sb(nx, ny, 24.0, 3, pw.shape[0], rep, cf) == EINVAL
    high = np.array([[13, 0]], np.int32)
    assert sb(nx, ny, 24.0, 1, 1, high, np.ones((1, 1))) == EUNSUP
    assert L.ash_set_precision(h, 7) == EINVAL
    # a valid set-up
    amp = torch.rand((ny, nx), dtype=torch.float32, device="cuda") + 0.1
    c.set_basis(nx, ny, modes=[1, 2, 4], amp=amp)
    c.set_spots(w)
    ph = (torch.rand((ny, nx), device="cuda") * 6.0 - 3.0).contiguous()
    E0 = c.forward(phase=ph).clone()
    # spot validation leaves the spots as they were
    wn = w.copy()
    wn[1, 2] = np.inf
    assert L.ash_set_spots(h, 4, wn.ctypes.data, None) == EINVAL
    assert L.ash_set_spots(h, 0, w.ctypes.data, None) == EINVAL
    t_bad = np.array([1.0, 0.0, 1.0, 1.0], np.float32)
    assert L.ash_set_spots(h, 4, w.ctypes.data, t_bad.ctypes.data) == EINVAL
    # transforms and loops
    field = torch.zeros((ny, nx), dtype=torch.complex64, device="cuda")
    assert L.ash_forward(h, _p(ph), _p(field), _p(E)) == EINVAL
    assert L.ash_forward(h, None, None, _p(E)) == EINVAL
    assert L.ash_forward(h, _p(ph), None, None) == EINVAL
    y = torch.ones(4, dtype=torch.complex64, device="cuda")
    assert L.ash_adjoint(h, _p(y), None, None) == EINVAL
    W = torch.ones(4, dtype=torch.float32, device="cuda")
    params = _lib.WgsParams(1.0, 0)
    assert L.ash_wgs_iterate(h, _p(ph), _p(W), -1, ctypes.byref(params), None,
                             None) == EINVAL
    params_nan = _lib.WgsParams(float("nan"), 0)
    assert L.ash_wgs_iterate(h, _p(ph), _p(W), 1, ctypes.byref(params_nan),
                             None, None) == EINVAL
    params_fix = _lib.WgsParams(1.0, -1)
    assert L.ash_wgs_iterate(h, _p(ph), _p(W), 1, ctypes.byref(params_fix),
                             None, None) == ENOTREADY
    assert L.ash_wgs_feedback(h, _p(ph), _p(W), None, ctypes.byref(params),
                              None, None) == EINVAL
    S = torch.empty(2, dtype=torch.float32, device="cuda")
    assert L.ash_window_strehl(h, _p(ph), 2, 3, _p(S)) == ESHAPE
    assert L.ash_get_fixed_phases(h, _p(S)) == ENOTREADY
    assert L.ash_coef_grad(h, _p(ph), None, _p(S)) == EINVAL
    # nothing above changed the context
    E1 = c.forward(phase=ph)
    assert torch.equal(E0, E1)
    _say("  last error:", L.ash_last_error(h).decode())
    c.close()


def _small_set(A, nx, ny, N, seed):
    rng = np.random.default_rng(seed)
    w = rng.normal(0, 0.5, size=(N, 3))
    w[:, 0] = np.pi * rng.uniform(-0.4 * ny, 0.4 * ny, N) * (min(nx, ny) / 2) / ny
    w[:, 1] = np.pi * rng.uniform(-0.4 * nx, 0.4 * nx, N) * (min(nx, ny) / 2) / nx
    amp = torch.tensor(rng.uniform(0.2, 1.0, size=(ny, nx)), dtype=torch.float32,
                       device="cuda")
    ph = torch.tensor(rng.uniform(-np.pi, np.pi, size=(ny, nx)),
                      dtype=torch.float32, device="cuda")
    return w, amp, ph


def test_injected_allocation_failures(A):
    """Device allocations made to fail (ash_inject_failure) return ASH_ENOMEM
    from the set-up calls and from batch creation; the objects stay valid,
    and repeating the calls gives bitwise the results of a context that
    never failed."""
    from paper_2505_08777_amd import _lib
    nx, ny, modes = 96, 64, [1, 2, 4]
    w, amp, ph = _small_set(A, nx, ny, 40, 11)
    ref = A.Context(0)
    ref.set_basis(nx, ny, modes=modes, amp=amp)
    ref.set_spots(w)
    E_ref = ref.forward(phase=ph).clone()
    c = A.Context(0)
    try:
        A.inject_failure(A.INJECT_ALLOC, 1)
        with pytest.raises(A.AshError) as ei:
            c.set_basis(nx, ny, modes=modes, amp=amp)
        assert ei.value.code == _lib.ENOMEM and "injected" in str(ei.value)
        _say("  ", ei.value)
        c.set_basis(nx, ny, modes=modes, amp=amp)
        A.inject_failure(A.INJECT_ALLOC, 1)
        with pytest.raises(A.AshError) as ei:
            c.set_spots(w)
        assert ei.value.code == _lib.ENOMEM
        c.set_spots(w)
        assert torch.equal(c.forward(phase=ph), E_ref)
        A.inject_failure(A.INJECT_ALLOC, 1)
        with pytest.raises(A.AshError) as ei:
            A.Batch([c, ref])
        assert ei.value.code == _lib.ENOMEM
        b = A.Batch([c, ref])
        b.set_form(False)  # per-hologram work units: equal members, equal bits
        phs = [ph.clone(), ph.clone()]
        b.wgs(phs, 2)
        assert torch.equal(phs[0], phs[1])
        # the one-launch form's pinned flag: its failure comes before any
        # launch (the phases are untouched), and the next call runs
        b.set_form(True)
        A.inject_failure(A.INJECT_ALLOC, 1)
        p_fail = [ph.clone(), ph.clone()]
        with pytest.raises(A.AshError) as ei:
            b.wgs(p_fail, 2)
        assert ei.value.code == _lib.ENOMEM
        assert torch.equal(p_fail[0], ph) and torch.equal(p_fail[1], ph)
        p_a, p_b = [ph.clone(), ph.clone()], [ph.clone(), ph.clone()]
        b.wgs(p_a, 2)
        b.wgs(p_b, 2)
        assert all(torch.equal(x, y) for x, y in zip(p_a, p_b))
        d = torch.remainder(p_a[0] - phs[0] + math.pi, 2 * math.pi) - math.pi
        assert d.abs().median().item() < 1e-4  # the per-phase form's step
        b.close()
    finally:
        A.inject_failure(A.INJECT_ALLOC, 0)
    c.close()
    ref.close()


def test_injected_barrier_failure(A):
    """A one-launch batch call whose barriers give up (their error flag set
    from the host before the launch, so nothing waits) returns ASH_EHIP
    with the barrier's message; the batch stays usable, and its next call
    equals bitwise a batch that never failed."""
    from paper_2505_08777_amd import _lib
    sizes = [(96, 64, 40, 21), (64, 64, 7, 22), (128, 96, 90, 23)]
    ctxs, starts = [], []
    for nx, ny, N, seed in sizes:
        w, amp, ph = _small_set(A, nx, ny, N, seed)
        c = A.Context(0)
        c.set_basis(nx, ny, modes=[1, 2, 4], amp=amp)
        c.set_spots(w)
        ctxs.append(c)
        starts.append(ph)
    clean = A.Batch(ctxs)
    clean.set_form(True)
    ph_c = [p.clone() for p in starts]
    W_c = [torch.ones(n, device="cuda") for _, _, n, _ in sizes]
    clean.wgs(ph_c, 3, weights=W_c)
    b = A.Batch(ctxs)
    b.set_form(True)
    try:
        A.inject_failure(A.INJECT_BARRIER, 1)
        with pytest.raises(A.AshError) as ei:
            b.wgs([p.clone() for p in starts], 3,
                  weights=[torch.ones(n, device="cuda") for _, _, n, _ in sizes])
        assert ei.value.code == _lib.EHIP and "barrier" in str(ei.value)
        _say("  ", ei.value)
    finally:
        A.inject_failure(A.INJECT_BARRIER, 0)
    ph_b = [p.clone() for p in starts]
    W_b = [torch.ones(n, device="cuda") for _, _, n, _ in sizes]
    b.wgs(ph_b, 3, weights=W_b)
    for x, y in zip(ph_b + W_b, ph_c + W_c):
        assert torch.equal(x, y)
    b.close()
    clean.close()
    for c in ctxs:
        c.close()
