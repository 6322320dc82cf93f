"""GPU parity of the differentiable form against the FP64 oracle.

The phase gradient behind the autograd Function, checked against the
oracle's analytic gradient and its central differences; one Adam update of
the on-device descent from an oracle state; and the full 1024 x 1024 /
1000-spot gradient on sampled pixels.
"""

import math
import sys

import numpy as np
import pytest

import oracle
import workloads
from tolerance import (GRAD_REL, GRAD_FD_REL, PHASE_RAD, assert_fields,
                       field_errors)

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


def _case(nx=96, ny=80, N=30, seed=41, modes=(1, 2, 3, 4, 5, 7, 12)):
    rng = np.random.default_rng(seed)
    geom = oracle.Geometry(nx, ny)
    basis = oracle.ZernikeBasis(list(modes))
    w = rng.normal(0, 0.6, size=(N, len(modes)))
    w[:, 0] = np.pi * rng.uniform(-0.4 * ny, 0.4 * ny, N) * geom.R / ny
    w[:, 1] = np.pi * rng.uniform(-0.4 * nx, 0.4 * nx, N) * geom.R / nx
    amp = rng.uniform(0.2, 1.0, size=(ny, nx)).astype(np.float32).astype(np.float64)
    t = rng.uniform(0.5, 1.0, size=N).astype(np.float32).astype(np.float64)
    phi = rng.uniform(-np.pi, np.pi, size=(ny, nx)).astype(np.float32).astype(np.float64)
    return rng, geom, basis, list(modes), w, amp, t, phi


def _ctx(A, geom, modes, w, amp, t):
    c = A.Context(0)
    c.set_basis(geom.nx, geom.ny, modes=modes,
                amp=torch.tensor(amp, dtype=torch.float32, device="cuda"))
    c.set_spots(w, t)
    return c


def test_phase_grad_matches_oracle(A):
    rng, geom, basis, modes, w, amp, t, phi = _case()
    G = (rng.normal(size=len(t)) + 1j * rng.normal(size=len(t))).astype(np.complex64)
    c = _ctx(A, geom, modes, w, amp, t)
    g = c.phase_grad(torch.tensor(phi, dtype=torch.float32, device="cuda"),
                     torch.tensor(G, device="cuda")).cpu().numpy()
    f = amp * np.exp(1j * phi)
    ref = np.imag(np.conj(f) * oracle.adjoint(G.astype(np.complex128), w, basis, geom))
    _say("phase_grad", field_errors(g, ref))
    assert_fields(g, ref, rel=GRAD_REL, what="phase gradient")
    c.close()


def test_autograd_function_loss_gradient_and_fd(A):
    rng, geom, basis, modes, w, amp, t, phi = _case(seed=42)
    c = _ctx(A, geom, modes, w, amp, t)
    s = oracle.spot_norm(amp, len(t))
    ph = torch.tensor(phi, dtype=torch.float32, device="cuda", requires_grad=True)
    E = A.propagate(ph, c)
    tt = torch.tensor(t, dtype=torch.float32, device="cuda")
    L = torch.sum((torch.abs(E / s) ** 2 - tt) ** 2)
    L.backward()
    g = ph.grad.cpu().numpy()
    ref, Lref, Eref = oracle.loss_grad(phi, amp, t, w, basis, geom, lam=0.0)
    _say("loss", float(L), Lref, "grad", field_errors(g, ref))
    assert abs(float(L) - Lref) <= 1e-4 * abs(Lref)
    assert_fields(E.detach().cpu().numpy(), Eref, what="forward")
    assert_fields(g, ref, rel=GRAD_REL, what="loss gradient")
    pix = rng.choice(geom.P, size=64, replace=False)
    fd = oracle.fd_grad(phi, pix, amp, t, w, basis, geom, h=1e-4, lam=0.0, E=Eref)
    d = np.abs(g.reshape(-1)[pix] - fd)
    rms = np.sqrt(np.mean(fd ** 2))
    _say("fd", d.max() / rms)
    assert d.max() <= GRAD_FD_REL * rms
    c.close()


@pytest.mark.parametrize("lam", [1e-3, 300.0], ids=["tv1e-3", "tv-dominant"])
def test_adam_step_from_oracle_state(A, lam):
    # lam = 300 makes the TV term dominate the gradient, so the moments
    # check the TV derivative of the adjoint's epilogue as well
    rng, geom, basis, modes, w, amp, t, phi0 = _case(nx=130, ny=70, N=45, seed=43)
    lr, tv_eps = 0.05, 1e-3
    phi3, m3, v3, _ = oracle.adam_run(phi0, amp, t, w, basis, geom, 3, lr=lr,
                                      lam=lam, tv_eps=tv_eps)
    f32 = lambda a: np.asarray(a, np.float32).astype(np.float64)
    phi3, m3, v3 = f32(phi3), f32(m3), f32(v3)
    g, Lref, Eref = oracle.loss_grad(phi3, amp, t, w, basis, geom, lam=lam, eps=tv_eps)
    phi4, m4, v4 = oracle.adam_step(phi3, g, m3, v3, 4, lr=lr)
    c = _ctx(A, geom, modes, w, amp, t)
    cu = lambda a: torch.tensor(a, dtype=torch.float32, device="cuda")
    ph, m, v = cu(phi3), cu(m3), cu(v3)
    _, m, v, loss, E = c.adam(ph, 1, m=m, v=v, step0=3, lr=lr, tv_weight=lam,
                              tv_eps=tv_eps, want_E=True)
    _say("adam loss", float(loss[0]), Lref)
    assert abs(float(loss[0]) - Lref) <= 1e-4 * abs(Lref)
    assert_fields(E.cpu().numpy(), Eref, what="forward")
    # m is linear in the gradient; v in its square
    assert_fields(m.cpu().numpy(), m4, rel=GRAD_REL, what="first moment")
    assert_fields(v.cpu().numpy(), v4, rel=2 * GRAD_REL, what="second moment")
    d = np.abs(ph.cpu().numpy().astype(np.float64) - phi4)
    _say("adam phase", d.max())
    assert d.max() <= PHASE_RAD
    c.close()


def test_adam_descends(A):
    rng, geom, basis, modes, w, amp, t, phi0 = _case(nx=128, ny=64, N=20, seed=44)
    c = _ctx(A, geom, modes, w, amp, t)
    ph = torch.tensor(phi0, dtype=torch.float32, device="cuda")
    _, m, v, loss, _ = c.adam(ph, 40, lr=0.05)
    L = loss.cpu().numpy()
    _say("losses", L[0], L[10], L[-1])
    assert np.all(np.isfinite(L)) and L[-1] < 0.5 * L[0]
    # continuing from the returned moments equals one longer run
    ph2 = torch.tensor(phi0, dtype=torch.float32, device="cuda")
    _, m2, v2, l2, _ = c.adam(ph2, 20, lr=0.05)
    _, m2, v2, l3, _ = c.adam(ph2, 20, m=m2, v=v2, step0=20, lr=0.05)
    assert torch.equal(ph, ph2)
    np.testing.assert_array_equal(np.concatenate([l2.cpu().numpy(), l3.cpu().numpy()]), L)
    c.close()


def test_grad1024_sampled_gradient(A):
    """The full differentiable workload (1024 x 1024, 1000 spots): the
    gradient at the start phase on 4096 sampled pixels against the oracle,
    and at 64 of them against FP64 central differences."""
    d = workloads.grad1024()
    geom = oracle.Geometry(d["nx"], d["ny"])
    basis = oracle.ZernikeBasis(d["modes"])
    amp = d["amp"].astype(np.float32).astype(np.float64)
    phi = d["phi0"].astype(np.float32).astype(np.float64)
    t = d["t"].astype(np.float32).astype(np.float64)
    c = _ctx(A, geom, d["modes"], d["w"], amp, t)
    ph = torch.tensor(phi, dtype=torch.float32, device="cuda", requires_grad=True)
    E = A.propagate(ph, c)
    s = oracle.spot_norm(amp, len(t))
    L = torch.sum((torch.abs(E / s) ** 2 - torch.tensor(t, dtype=torch.float32, device="cuda")) ** 2)
    L.backward()
    g = ph.grad.cpu().numpy().reshape(-1)
    rng = np.random.default_rng(45)
    pix = np.sort(rng.choice(geom.P, size=4096, replace=False))
    Eref = oracle.forward(amp * np.exp(1j * phi), d["w"], basis, geom)
    assert_fields(E.detach().cpu().numpy(), Eref, what="forward")
    Eh = Eref / s
    G = 4.0 * (np.abs(Eh) ** 2 - t) * Eh / s
    h = oracle.adjoint(G, d["w"], basis, geom, pixels=pix)
    ref = np.imag(np.conj((amp * np.exp(1j * phi)).reshape(-1)[pix]) * h)
    _say("grad1024", field_errors(g[pix], ref))
    assert_fields(g[pix], ref, rel=GRAD_REL, what="sampled gradient")
    fdp = pix[:64]
    fd = oracle.fd_grad(phi, fdp, amp, t, d["w"], basis, geom, h=1e-4, lam=0.0, E=Eref)
    dd = np.abs(g[fdp] - fd)
    _say("grad1024 fd", dd.max() / np.sqrt(np.mean(fd ** 2)))
    assert dd.max() <= GRAD_FD_REL * np.sqrt(np.mean(fd ** 2))
    c.close()
