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
