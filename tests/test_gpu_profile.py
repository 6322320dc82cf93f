"""Event timing through the C ABI: only the selected categories are timed,
one launch in every `stride` of each, the read clears the record, and
timing changes no result."""

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


def test_profile_stride_and_categories(A):
    from paper_2505_08777_amd import _lib
    nx, ny, N = 96, 64, 40
    c = A.Context(0)
    amp = torch.rand((ny, nx), dtype=torch.float32, device="cuda") + 0.1
    c.set_basis(nx, ny, modes=[1, 2, 4, 12], amp=amp)
    c.set_spots(np.random.default_rng(3).normal(scale=2.0, size=(N, 4)))
    ph = (torch.rand((ny, nx), device="cuda") * 6.0 - 3.0).contiguous()
    y = torch.ones(N, dtype=torch.complex64, device="cuda")
    E0 = c.forward(phase=ph).clone()
    g0 = c.adjoint(y, field=True).clone()
    torch.cuda.synchronize()
    for stride, calls in ((1, 5), (4, 10), (3, 3)):
        c.profile(True, categories=("forward",), stride=stride)
        for _ in range(calls):
            E = c.forward(phase=ph)
            g = c.adjoint(y, field=True)
            assert torch.equal(E, E0) and torch.equal(g, g0)
        rec = c.profile_read()
        _say("  stride", stride, rec)
        assert rec["forward"][1] == (calls + stride - 1) // stride
        assert rec["forward"][0] > 0.0
        assert rec["adjoint"] == (0.0, 0)
        assert c.profile_read()["forward"] == (0.0, 0)    # read clears
    c.profile(False)
    c.forward(phase=ph)
    assert c.profile_read()["forward"] == (0.0, 0)
    assert _lib.lib.ash_profile_stride(c._h, 0) == _lib.EINVAL
    c.close()
