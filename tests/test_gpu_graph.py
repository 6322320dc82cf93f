"""The compute calls in a HIP graph: none of them allocates, synchronises or
records a memset, so a caller can capture them (here through torch's graph
capture on the context's stream) and replay them.  Each replay, with eager
work between replays, must equal the eager calls bitwise."""

import sys

import numpy as np
import pytest

import workloads

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


def test_wgs_and_transforms_replay_bitwise(A):
    d = workloads.plain256()
    dev = "cuda"
    c = A.Context(0)
    c.set_basis(d["nx"], d["ny"], modes=d["modes"],
                amp=torch.tensor(d["amp"], dtype=torch.float32, device=dev))
    c.set_spots(d["w"], d["t"])
    N = d["w"].shape[0]
    start = torch.tensor(d["phi0"], dtype=torch.float32, device=dev)
    ph = start.clone()
    W = torch.ones(N, dtype=torch.float32, device=dev)
    E = torch.empty(N, dtype=torch.complex64, device=dev)
    g_out = torch.empty((d["ny"], d["nx"]), dtype=torch.complex64, device=dev)
    y = torch.ones(N, dtype=torch.complex64, device=dev)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):           # warm-up on the capture stream
        c.wgs(ph, 5, weights=W, want_E=False, want_stats=False)
        c.forward(phase=ph, out=E)
    torch.cuda.current_stream().wait_stream(side)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        c.wgs(ph, 5, weights=W, want_E=False, want_stats=False)
        c.forward(phase=ph, out=E)
        g = c.adjoint(y, field=True)
        g_out.copy_(g)
    for rep in range(3):
        ph.copy_(start)
        W.fill_(1.0)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        pe = start.clone()
        We = torch.ones(N, dtype=torch.float32, device=dev)
        c.wgs(pe, 5, weights=We, want_E=False, want_stats=False)
        Ee = c.forward(phase=pe)
        ge = c.adjoint(y, field=True)
        torch.cuda.synchronize()
        _say("  replay", rep)
        assert torch.equal(ph, pe) and torch.equal(W, We)
        assert torch.equal(E, Ee) and torch.equal(g_out, ge)
    c.close()


def test_adam_and_coefficient_gradient_replay_bitwise(A):
    """The on-device Adam descent, the moment transform and the gradient in
    the coefficients captured once (after the usual warm-up on a side
    stream) and replayed, each replay equal to an eager run of the same
    calls bitwise."""
    nx, ny, N = 128, 96, 40
    modes = [1, 2, 3, 4, 5, 7, 12]
    rng = np.random.default_rng(77)
    dev = "cuda"
    w = rng.normal(0, 0.6, size=(N, len(modes)))
    w[:, 0] = np.pi * rng.uniform(-0.4 * ny, 0.4 * ny, N) * 48 / ny
    w[:, 1] = np.pi * rng.uniform(-0.4 * nx, 0.4 * nx, N) * 48 / nx
    t = rng.uniform(0.5, 1.0, N)
    c = A.Context(0)
    c.set_basis(nx, ny, modes=modes,
                amp=torch.rand((ny, nx), device=dev, dtype=torch.float32) + 0.2)
    c.set_spots(w, t)
    start = (torch.rand((ny, nx), device=dev) * 6.0 - 3.0).contiguous()
    G = torch.tensor(rng.normal(size=N) + 1j * rng.normal(size=N),
                     dtype=torch.complex64, device=dev)
    ph = start.clone()
    m = torch.zeros((ny, nx), dtype=torch.float32, device=dev)
    v = torch.zeros_like(m)
    cg = torch.empty((N, len(modes)), dtype=torch.float32, device=dev)
    mo = torch.empty((N, len(modes)), dtype=torch.complex64, device=dev)

    def work(p, mm, vv, cg_out, mo_out):
        _, _, _, loss, _ = c.adam(p, 3, m=mm, v=vv)
        c.coef_grad(p, G, out=cg_out)
        c.forward_moments(p, out=mo_out)
        return loss

    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        work(start.clone(), torch.zeros_like(m), torch.zeros_like(m),
             torch.empty_like(cg), torch.empty_like(mo))
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        loss_g = work(ph, m, v, cg, mo)
    for rep in range(3):
        ph.copy_(start)
        m.zero_()
        v.zero_()
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        pe, me, ve = start.clone(), torch.zeros_like(m), torch.zeros_like(m)
        cge, moe = torch.empty_like(cg), torch.empty_like(mo)
        loss_e = work(pe, me, ve, cge, moe)
        torch.cuda.synchronize()
        _say("  replay", rep, float(loss_g[-1]))
        assert torch.equal(ph, pe) and torch.equal(m, me) and torch.equal(v, ve)
        assert torch.equal(loss_g, loss_e)
        assert torch.equal(cg, cge) and torch.equal(mo, moe)
    c.close()
