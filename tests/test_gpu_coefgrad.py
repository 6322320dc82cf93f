"""GPU parity of the basis moments of the forward and of the gradient with
respect to the kernel coefficients (ash_forward_moments, ash_coef_grad,
PropagateSpots) against the FP64 oracle.

Each moment column d is held to the field bar on its own (elementwise with
the column's rms floor, and normwise), since the columns' scales differ with
the size of Z_d.
"""

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


def _spots(rng, nx, ny, N, modes, sigma, R, tilt_scale=1.0):
    w = rng.normal(0, sigma, size=(N, len(modes)))
    if 1 in modes:
        w[:, modes.index(1)] = tilt_scale * np.pi * rng.uniform(-ny / 2, ny / 2, N) * R / ny
    if 2 in modes:
        w[:, modes.index(2)] = tilt_scale * np.pi * rng.uniform(-nx / 2, nx / 2, N) * R / nx
    return w


def _assert_columns(M, Mref, what):
    worst = (0.0, 0.0)
    for d in range(M.shape[1]):
        per, norm = assert_fields(M[:, d], Mref[:, d], what="%s column %d" % (what, d))
        worst = (max(worst[0], per), max(worst[1], norm))
    return worst


# (nx, ny, N, ANSI modes, sigma, R, tilt scale)
CASES = [
    (256, 256, 25, [1, 2, 3, 4, 5, 6, 7, 8, 9, 12], 0.5, None, 1.0),
    (100, 37, 70, [0, 1, 2, 4, 7, 12], 1.0, 50.0, 1.0),       # ragged tiles
    (200, 120, 130, list(range(15)), 0.8, 100.0, 1.0),         # 15 modes
    (130, 70, 200, list(range(21)), 0.5, 65.0, 1.0),           # 2D > 32 rows
    (33, 1, 5, [2, 3, 5], 1.0, 16.5, 1.0),                     # single row
    (96, 80, 45, [1, 2, 4, 7], 0.7, None, 9.0),                # range reduction
]


@pytest.mark.parametrize("nx,ny,N,modes,sigma,R,ts", CASES)
def test_moments_and_coef_grad_parity(A, nx, ny, N, modes, sigma, R, ts):
    _say("case", nx, ny, N, modes, sigma, R, ts)
    rng = np.random.default_rng(nx * 7 + ny + N)
    geom = oracle.Geometry(nx, ny, R=R)
    basis = oracle.ZernikeBasis(modes)
    w = _spots(rng, nx, ny, N, modes, sigma, geom.R, ts)
    amp = rng.uniform(0.2, 1.0, size=(ny, nx)).astype(np.float32).astype(np.float64)
    phi = rng.uniform(-np.pi, np.pi, size=(ny, nx)).astype(np.float32).astype(np.float64)
    c = A.Context(0)
    c.set_basis(nx, ny, modes=modes, R=geom.R,
                amp=torch.tensor(amp, dtype=torch.float32, device="cuda"))
    c.set_spots(w)
    _say("  info", c.info())
    ph = torch.tensor(phi, dtype=torch.float32, device="cuda")
    M = c.forward_moments(ph).cpu().numpy()
    f = amp * np.exp(1j * phi)
    Mref = oracle.forward_moments(f, w, basis, geom)
    _say("  moments", _assert_columns(M, Mref, "moments"))
    G = (rng.normal(size=N) + 1j * rng.normal(size=N)).astype(np.complex64)
    g = c.coef_grad(ph, torch.tensor(G, device="cuda")).cpu().numpy()
    gref = oracle.coef_grad(f, w, basis, geom, G.astype(np.complex128))
    _say("  coef grad", field_errors(g, gref))
    assert_fields(g, gref, what="coefficient gradient")
    c.close()


def test_autograd_in_coefficients_and_phase(A):
    """PropagateSpots: torch's gradients of a spot-amplitude loss in w and
    in the phase against the oracle's analytic gradients."""
    nx, ny, N, modes = 128, 96, 60, [1, 2, 3, 4, 5, 6, 7, 8, 9, 12]
    rng = np.random.default_rng(5)
    geom = oracle.Geometry(nx, ny)
    basis = oracle.ZernikeBasis(modes)
    w = _spots(rng, nx, ny, N, modes, 0.5, geom.R)
    amp = rng.uniform(0.2, 1.0, size=(ny, nx)).astype(np.float32).astype(np.float64)
    phi = rng.uniform(-np.pi, np.pi, size=(ny, nx)).astype(np.float32).astype(np.float64)
    t = rng.uniform(0.5, 1.0, N)
    c = A.Context(0)
    c.set_basis(nx, ny, modes=modes,
                amp=torch.tensor(amp, dtype=torch.float32, device="cuda"))
    c.set_spots(w)
    ph = torch.tensor(phi, dtype=torch.float32, device="cuda", requires_grad=True)
    wt = torch.tensor(w, dtype=torch.float64, requires_grad=True)
    E = A.propagate(ph, c, w=wt)
    s = oracle.spot_norm(amp, N)
    L = torch.sum((torch.abs(E / s) ** 2 - torch.tensor(t, dtype=torch.float32, device="cuda")) ** 2)
    L.backward()
    f = amp * np.exp(1j * phi)
    Eref = oracle.forward(f, w, basis, geom)
    Eh = Eref / s
    G = 4.0 * (np.abs(Eh) ** 2 - t) * Eh / s
    gw = oracle.coef_grad(f, w, basis, geom, G)
    _say("  dL/dw", field_errors(wt.grad.numpy(), gw))
    assert_fields(wt.grad.numpy(), gw, rel=1e-4, what="dL/dw")
    gp = np.imag(np.conj(f) * oracle.adjoint(G, w, basis, geom))
    _say("  dL/dphi", field_errors(ph.grad.cpu().numpy(), gp))
    assert_fields(ph.grad.cpu().numpy(), gp, rel=1e-4, what="dL/dphi")
    c.close()


def test_grad1024_sampled_moments(A):
    """The 1024 x 1024, 1000-spot workload: moments and the coefficient
    gradient of 16 sampled spots against the oracle."""
    d = workloads.grad1024()
    nx, ny, N = d["nx"], d["ny"], d["w"].shape[0]
    geom = oracle.Geometry(nx, ny)
    basis = oracle.ZernikeBasis(d["modes"])
    amp = d["amp"].astype(np.float32).astype(np.float64)
    phi = d["phi0"].astype(np.float32).astype(np.float64)
    c = A.Context(0)
    c.set_basis(nx, ny, modes=d["modes"],
                amp=torch.tensor(d["amp"], dtype=torch.float32, device="cuda"))
    c.set_spots(d["w"], d["t"])
    _say("  info", c.info())
    ph = torch.tensor(phi, dtype=torch.float32, device="cuda")
    M = c.forward_moments(ph).cpu().numpy()
    rng = np.random.default_rng(16)
    sel = np.sort(rng.choice(N, size=16, replace=False))
    f = amp * np.exp(1j * phi)
    Mref = oracle.forward_moments(f, d["w"], basis, geom, spots=sel)
    _say("  moments", field_errors(M[sel], Mref))
    # the sampled rows are too few for a per-column rms floor: hold the
    # whole sample to the field bar
    assert_fields(M[sel], Mref, what="sampled moments")
    G = (rng.normal(size=N) + 1j * rng.normal(size=N)).astype(np.complex64)
    g = c.coef_grad(ph, torch.tensor(G, device="cuda")).cpu().numpy()
    gref = oracle.coef_grad(f, d["w"], basis, geom, G[sel].astype(np.complex128), spots=sel)
    _say("  coef grad", field_errors(g[sel], gref))
    assert_fields(g[sel], gref, what="sampled coefficient gradient")
    c.close()


def test_backward_after_spot_change(A):
    """Two propagate calls with different w before one backward: each
    backward uses its own forward's spots (PropagateSpots sets them back),
    and a phase-only propagate whose context changed spots refuses."""
    nx, ny, N, modes = 96, 64, 40, [1, 2, 3, 4, 5, 6]
    rng = np.random.default_rng(77)
    geom = oracle.Geometry(nx, ny)
    basis = oracle.ZernikeBasis(modes)
    w1 = _spots(rng, nx, ny, N, modes, 0.5, geom.R)
    w2 = _spots(rng, nx, ny, N, modes, 0.5, geom.R)
    amp = rng.uniform(0.2, 1.0, size=(ny, nx)).astype(np.float32).astype(np.float64)
    phi = rng.uniform(-np.pi, np.pi, size=(ny, nx)).astype(np.float32).astype(np.float64)
    G = (rng.normal(size=N) + 1j * rng.normal(size=N)).astype(np.complex64)
    c = A.Context(0)
    c.set_basis(nx, ny, modes=modes,
                amp=torch.tensor(amp, dtype=torch.float32, device="cuda"))
    c.set_spots(w1)
    Gt = torch.tensor(G, device="cuda")
    ph1 = torch.tensor(phi, dtype=torch.float32, device="cuda", requires_grad=True)
    ph2 = torch.tensor(phi, dtype=torch.float32, device="cuda", requires_grad=True)
    wt1 = torch.tensor(w1, dtype=torch.float64, requires_grad=True)
    wt2 = torch.tensor(w2, dtype=torch.float64, requires_grad=True)
    E1 = A.propagate(ph1, c, w=wt1)
    E2 = A.propagate(ph2, c, w=wt2)      # the context now holds w2
    # L = Re(sum conj(G) E) has field gradient G
    torch.sum(torch.real(torch.conj(Gt) * E1)).backward()
    f = amp * np.exp(1j * phi)
    gw = oracle.coef_grad(f, w1, basis, geom, G.astype(np.complex128))
    gp = np.imag(np.conj(f) * oracle.adjoint(G.astype(np.complex128), w1, basis, geom))
    _say("  first backward: dL/dw", field_errors(wt1.grad.numpy(), gw),
         "dL/dphi", field_errors(ph1.grad.cpu().numpy(), gp))
    assert_fields(wt1.grad.numpy(), gw, what="dL/dw of the first forward")
    assert_fields(ph1.grad.cpu().numpy(), gp, what="dL/dphi of the first forward")
    torch.sum(torch.real(torch.conj(Gt) * E2)).backward()
    gw2 = oracle.coef_grad(f, w2, basis, geom, G.astype(np.complex128))
    assert_fields(wt2.grad.numpy(), gw2, what="dL/dw of the second forward")
    # phase-only propagate: a set_spots between forward and backward refuses
    ph3 = torch.tensor(phi, dtype=torch.float32, device="cuda", requires_grad=True)
    E3 = A.propagate(ph3, c)
    c.set_spots(w1)
    with pytest.raises(RuntimeError):
        torch.sum(torch.real(torch.conj(Gt) * E3)).backward()
    c.close()
