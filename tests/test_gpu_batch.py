"""GPU parity of the batched form.

Each hologram of a batch against the same hologram run alone on the GPU
(same kernels, other partial-sum grouping: equal to FP32 summation order)
and against the FP64 oracle's WGS step; the autotuner and its table; the
invalidation of a batch whose member changed; and the full 64-hologram
workload on its smallest holograms.
"""

import os
import sys

import numpy as np
import pytest

import oracle
import workloads
from tolerance import (PHASE_RAD, STEP_PHASE_MASK, assert_phase, field_errors)

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


# (nx, ny, N, ANSI modes, sigma, tilt scale, full precision): mixed sizes,
# ragged tiles, one spot, 3-piece and range-reduced record shapes
SPECS = [
    (96, 80, 30, [1, 2, 3, 4, 5, 7, 12], 0.6, 1.0, False),
    (130, 70, 45, [1, 2, 3, 4, 5, 6, 7, 8, 9, 12], 0.5, 1.0, False),
    (64, 64, 1, [1, 2, 4], 0.3, 1.0, False),
    (200, 120, 130, [1, 2, 3, 4, 5, 6, 7, 8, 9, 12], 0.5, 1.0, True),
    (48, 40, 70, [1, 2, 4, 7], 0.7, 9.0, False),
    (33, 1, 5, [2, 3, 5], 1.0, 1.0, False),
]


def _holo(spec, seed):
    nx, ny, N, modes, sigma, tilt, full = spec
    rng = np.random.default_rng(seed)
    geom = oracle.Geometry(nx, ny)
    w = rng.normal(0, sigma, size=(N, len(modes)))
    if 1 in modes:
        w[:, modes.index(1)] = tilt * np.pi * rng.uniform(-ny / 2, ny / 2, N) * geom.R / ny
    if 2 in modes:
        w[:, modes.index(2)] = tilt * np.pi * rng.uniform(-nx / 2, nx / 2, N) * geom.R / nx
    amp = rng.uniform(0.2, 1.0, size=(ny, nx)).astype(np.float32).astype(np.float64)
    t = rng.uniform(0.5, 1.0, size=N).astype(np.float32).astype(np.float64)
    phi = rng.uniform(-np.pi, np.pi, size=(ny, nx)).astype(np.float32).astype(np.float64)
    return dict(nx=nx, ny=ny, modes=modes, w=w, amp=amp, t=t, phi=phi, full=full,
                geom=geom)


def _ctx(A, h):
    c = A.Context(0)
    c.set_precision(h["full"])
    c.set_basis(h["nx"], h["ny"], modes=h["modes"],
                amp=torch.tensor(h["amp"], dtype=torch.float32, device="cuda"))
    c.set_spots(h["w"], h["t"])
    return c


def _cu(a):
    return torch.tensor(np.asarray(a), dtype=torch.float32, device="cuda")


@pytest.fixture(scope="module")
def batch_case(A):
    holos = [_holo(s, 600 + i) for i, s in enumerate(SPECS)]
    ctxs = [_ctx(A, h) for h in holos]
    yield holos, ctxs
    for c in ctxs:
        c.close()


def test_batch_shapes(A, batch_case):
    holos, ctxs = batch_case
    infos = [c.info() for c in ctxs]
    _say([(i["groups"], i["range_reduce"]) for i in infos])
    b = A.Batch(ctxs)
    inf = b.info()
    _say(inf)
    shapes = {(i["groups"], i["range_reduce"]) for i in infos}
    assert inf["holograms"] == len(ctxs) and inf["shapes"] == len(shapes) >= 3
    assert inf["evals_per_transform"] == sum(h["w"].shape[0] * h["nx"] * h["ny"]
                                             for h in holos)
    b.close()


@pytest.mark.parametrize("n_iter", [1, 3])
def test_batch_equals_unbatched(A, batch_case, n_iter):
    holos, ctxs = batch_case
    b = A.Batch(ctxs)
    ph_b = [_cu(h["phi"]) for h in holos]
    W_b = [torch.ones(h["w"].shape[0], device="cuda") for h in holos]
    b.wgs(ph_b, n_iter, weights=W_b)
    torch.cuda.synchronize()
    for h, c, pb, wb in zip(holos, ctxs, ph_b, W_b):
        ph = _cu(h["phi"])
        _, W, E, _ = c.wgs(ph, n_iter)
        # conditioning mask from the unbatched path's last projection
        y = (W * _cu(h["t"])).to(torch.complex64) * E / E.abs().clamp_min(1e-30)
        g = c.adjoint(y.to(torch.complex64)).cpu().numpy()
        # each iteration adds its own rounding difference (the forward's
        # partial sums run over ranges of different lengths), as for the
        # weights below: 1e-4 rad per iteration
        err = assert_phase(pb.cpu().numpy(), ph.cpu().numpy(), g,
                           bar=1e-4 * n_iter, mask=STEP_PHASE_MASK,
                           what="batch vs alone")
        _say("holo", h["nx"], h["ny"], h["w"].shape[0], "phase", err)
        np.testing.assert_allclose(wb.cpu().numpy(), W.cpu().numpy(),
                                   rtol=1e-5 * n_iter, atol=1e-6)
    b.close()


def test_batch_step_matches_oracle(A, batch_case):
    holos, ctxs = batch_case
    b = A.Batch(ctxs)
    ph_b = [_cu(h["phi"]) for h in holos]
    W_b = [torch.ones(h["w"].shape[0], device="cuda") for h in holos]
    b.wgs(ph_b, 1, weights=W_b)
    for h, pb, wb in zip(holos, ph_b, W_b):
        basis = oracle.ZernikeBasis(h["modes"])
        N = h["w"].shape[0]
        ref_phi, ref_W, ref_E, _ = oracle.wgs_step(h["phi"], np.ones(N), h["t"], h["amp"],
                                                   h["w"], basis, h["geom"])
        np.testing.assert_allclose(wb.cpu().numpy(), ref_W, rtol=2e-4)
        a = np.abs(ref_E)
        y = ref_W * h["t"] * np.where(a > 0, ref_E / np.where(a > 0, a, 1), 1)
        gref = oracle.adjoint(y, h["w"], basis, h["geom"])
        _say("holo", h["nx"], h["ny"], N, assert_phase(
            pb.cpu().numpy(), ref_phi, gref, mask=STEP_PHASE_MASK,
            what="batch step"))
    b.close()


def test_batch_tuning_table(A, batch_case, tmp_path):
    holos, ctxs = batch_case
    b = A.Batch(ctxs)
    ph = [_cu(h["phi"]) for h in holos]
    path = str(tmp_path / "tune.txt")
    inf = b.tune(ph, table_out=path)
    _say(inf, open(path).read())
    assert all(L in (16, 32, 64, 128, 256, 512) for L in inf["range_blocks"])
    rows = [l.split() for l in open(path) if not l.startswith("#")]
    assert len(rows) == inf["shapes"]
    b2 = A.Batch(ctxs)
    b2.load_tuning(path)
    assert b2.info()["range_blocks"] == inf["range_blocks"]
    # the tuned batch still computes the same step
    p1 = [_cu(h["phi"]) for h in holos]
    p2 = [_cu(h["phi"]) for h in holos]
    b.wgs(p1, 1)
    b2.wgs(p2, 1)
    for a, c in zip(p1, p2):
        assert torch.equal(a, c)
    b.close()
    b2.close()


def test_batch_rejects_changed_member(A):
    h = _holo(SPECS[0], 700)
    c = _ctx(A, h)
    b = A.Batch([c])
    c.set_spots(h["w"][:10], h["t"][:10])
    with pytest.raises(A.AshError):
        b.wgs([_cu(h["phi"])], 1)
    b.close()
    c.close()


def test_batch64_smallest_holograms(A):
    """The full 64-hologram workload, one batched iteration; its three
    smallest holograms (by N * P) against the oracle's WGS step."""
    holos = workloads.make("batch64")
    ctxs = []
    for d in holos:
        c = A.Context(0)
        c.set_basis(d["nx"], d["ny"], modes=d["modes"],
                    amp=torch.tensor(d["amp"], dtype=torch.float32, device="cuda"))
        c.set_spots(d["w"], d["t"])
        ctxs.append(c)
    b = A.Batch(ctxs)
    _say(b.info())
    ph = [_cu(d["phi0"]) for d in holos]
    W = [torch.ones(d["w"].shape[0], device="cuda") for d in holos]
    b.wgs(ph, 1, weights=W)
    torch.cuda.synchronize()
    order = np.argsort([d["w"].shape[0] * d["nx"] * d["ny"] for d in holos])
    rng = np.random.default_rng(64)
    for h in order[:3]:
        d = holos[h]
        geom = oracle.Geometry(d["nx"], d["ny"])
        basis = oracle.ZernikeBasis(d["modes"])
        amp = d["amp"].astype(np.float32).astype(np.float64)
        phi = d["phi0"].astype(np.float32).astype(np.float64)
        N = d["w"].shape[0]
        E = oracle.forward(amp * np.exp(1j * phi), d["w"], basis, geom)
        a = np.abs(E)
        r = (a / np.linalg.norm(a)) / (d["t"] / np.linalg.norm(d["t"]))
        Wr = 1.0 / r
        Wr /= Wr.mean()
        np.testing.assert_allclose(W[h].cpu().numpy(), Wr, rtol=2e-4)
        pix = np.sort(rng.choice(geom.P, size=4096, replace=False))
        g = oracle.adjoint(Wr * d["t"] * E / a, d["w"], basis, geom, pixels=pix)
        got = ph[h].cpu().numpy().reshape(-1)[pix]
        err = assert_phase(got, np.angle(g), g, mask=STEP_PHASE_MASK,
                           what="batch64 holo %d" % h)
        _say("batch64 holo", h, d["nx"], N, err)
    b.close()
    for c in ctxs:
        c.close()
