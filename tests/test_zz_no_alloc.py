"""The allocation-free forward (ash_forward_noalloc) against ash_forward.

It runs the same kernels with the partial sums in the library's static
device scratch, so its fields equal ash_forward's; they are checked to the
field bar (and reported bitwise) on two calls in a row, the second on a
smaller set-up than the first, and against the FP64 oracle on the small
one.  Sizes beyond the scratch are refused.
"""

import ctypes
import sys

import numpy as np
import pytest

import oracle
import workloads
from tolerance import assert_fields, field_errors

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


def _noalloc(A, ctx, phase=None, field=None):
    """E through the C ABI's ash_forward_noalloc."""
    from paper_2505_08777_amd import _lib
    E = torch.empty(ctx.N, dtype=torch.complex64, device="cuda")
    ctx._stream()
    p = ctypes.c_void_p(phase.data_ptr()) if phase is not None else None
    f = ctypes.c_void_p(field.data_ptr()) if field is not None else None
    _lib.check(_lib.lib.ash_forward_noalloc(ctx._h, p, f,
                                            ctypes.c_void_p(E.data_ptr())),
               "ash_forward_noalloc", ctx._h)
    return E


def _case(A, nx, ny, N, modes, seed):
    rng = np.random.default_rng(seed)
    geom = oracle.Geometry(nx, ny)
    w = rng.normal(0, 0.6, size=(N, len(modes)))
    w[:, modes.index(1)] = np.pi * rng.uniform(-ny / 2, ny / 2, N) * geom.R / ny
    w[:, modes.index(2)] = np.pi * rng.uniform(-nx / 2, nx / 2, N) * geom.R / nx
    amp = rng.uniform(0.2, 1.0, size=(ny, nx)).astype(np.float32).astype(np.float64)
    phi = rng.uniform(-np.pi, np.pi, size=(ny, nx)).astype(np.float32).astype(np.float64)
    c = A.Context(0)
    c.set_basis(nx, ny, modes=modes,
                amp=torch.tensor(amp, dtype=torch.float32, device="cuda"))
    c.set_spots(w)
    return c, w, amp, phi, geom


def test_noalloc_forward_matches_forward(A):
    d = workloads.field1024()
    c1 = A.Context(0)
    c1.set_basis(d["nx"], d["ny"], modes=d["modes"],
                 amp=torch.tensor(d["amp"], dtype=torch.float32, device="cuda"))
    c1.set_spots(d["w"], d["t"])
    _say("first call: 1024 x 1024, 400 spots", c1.info())
    ph1 = torch.tensor(d["phi0"], dtype=torch.float32, device="cuda")
    E_ref1 = c1.forward(phase=ph1).cpu().numpy()
    E_na1 = _noalloc(A, c1, phase=ph1).cpu().numpy()
    _say("  vs ash_forward", field_errors(E_na1, E_ref1),
         "bitwise", bool(np.array_equal(E_na1, E_ref1)))
    assert_fields(E_na1, E_ref1, what="noalloc vs forward (1024^2)")
    # second call: a smaller set-up (fewer spots, fewer ranges) reusing the
    # scratch, with a complex nearfield input
    modes = [1, 2, 3, 4, 5, 6, 7, 8, 9, 12]
    c2, w, amp, phi, geom = _case(A, 200, 120, 57, modes, 11)
    _say("second call: 200 x 120, 57 spots", c2.info())
    f = amp * np.exp(1j * phi)
    ft = torch.tensor(f.astype(np.complex64), device="cuda")
    E_ref2 = c2.forward(field=ft).cpu().numpy()
    E_na2 = _noalloc(A, c2, field=ft).cpu().numpy()
    _say("  vs ash_forward", field_errors(E_na2, E_ref2),
         "bitwise", bool(np.array_equal(E_na2, E_ref2)))
    assert_fields(E_na2, E_ref2, what="noalloc vs forward (200 x 120)")
    Eo = oracle.forward(f.astype(np.complex64).astype(np.complex128), w,
                        oracle.ZernikeBasis(modes), geom)
    _say("  vs oracle", field_errors(E_na2, Eo))
    assert_fields(E_na2, Eo, what="noalloc vs oracle")
    # the first set-up again, after the smaller call
    E_na3 = _noalloc(A, c1, phase=ph1).cpu().numpy()
    assert_fields(E_na3, E_ref1, what="noalloc vs forward, third call")
    c1.close()
    c2.close()


def test_noalloc_forward_refuses_oversized(A):
    from paper_2505_08777_amd import _lib
    # 2^20 spots on a small SLM: at least 8 forward ranges of 2^20 spots,
    # 64 MiB of partial sums
    nx = ny = 64
    N = 1 << 20
    rng = np.random.default_rng(3)
    modes = [1, 2, 4]
    w = rng.normal(0, 0.3, size=(N, 3))
    c = A.Context(0)
    c.set_basis(nx, ny, modes=modes)
    c.set_spots(w)
    ph = torch.zeros((ny, nx), dtype=torch.float32, device="cuda")
    E = torch.empty(N, dtype=torch.complex64, device="cuda")
    rc = _lib.lib.ash_forward_noalloc(c._h, ctypes.c_void_p(ph.data_ptr()),
                                      None, ctypes.c_void_p(E.data_ptr()))
    _say("oversized:", rc, _lib.lib.ash_last_error(c._h).decode())
    assert rc == _lib.EUNSUPPORTED
    # the context still works through the allocating entry point
    c.forward(phase=ph, out=E)
    torch.cuda.synchronize()
    c.close()
