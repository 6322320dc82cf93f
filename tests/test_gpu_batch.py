"""GPU parity of the batched form.

Each hologram of a batch against the same hologram run alone on the GPU
(same kernels, other partial-sum grouping: equal to FP32 summation order)
and against the FP64 oracle's WGS step; the autotuner and its table; the
invalidation of a batch whose member changed; and the full 64-hologram
workload on every member (against its unbatched run), its smallest members
(against the oracle's step) and its largest (sampled transforms).
"""

import os
import sys

import numpy as np
import pytest

import oracle
import stepcheck
import workloads
from tolerance import (FP32_SUM_REL, assert_fields, assert_step_phase,
                       assert_step_weights, field_errors, step_bars)

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


# (nx, ny, N, ANSI modes, sigma, tilt scale, full precision, pupil radius):
# mixed sizes, ragged tiles, one spot, 3-piece and range-reduced record
# shapes, a single row (pupil radius along the row)
SPECS = [
    (96, 80, 30, [1, 2, 3, 4, 5, 7, 12], 0.6, 1.0, False, None),
    (130, 70, 45, [1, 2, 3, 4, 5, 6, 7, 8, 9, 12], 0.5, 1.0, False, None),
    (64, 64, 1, [1, 2, 4], 0.3, 1.0, False, None),
    (200, 120, 130, [1, 2, 3, 4, 5, 6, 7, 8, 9, 12], 0.5, 1.0, True, None),
    (48, 40, 70, [1, 2, 4, 7], 0.7, 9.0, False, None),
    (33, 1, 5, [2, 3, 5], 1.0, 1.0, False, 16.5),
]


def _holo(spec, seed):
    nx, ny, N, modes, sigma, tilt, full, R = spec
    rng = np.random.default_rng(seed)
    geom = oracle.Geometry(nx, ny, R=R)
    w = rng.normal(0, sigma, size=(N, len(modes)))
    if 1 in modes:
        w[:, modes.index(1)] = tilt * np.pi * rng.uniform(-ny / 2, ny / 2, N) * geom.R / ny
    if 2 in modes:
        w[:, modes.index(2)] = tilt * np.pi * rng.uniform(-nx / 2, nx / 2, N) * geom.R / nx
    amp = rng.uniform(0.2, 1.0, size=(ny, nx)).astype(np.float32).astype(np.float64)
    t = rng.uniform(0.5, 1.0, size=N).astype(np.float32).astype(np.float64)
    phi = rng.uniform(-np.pi, np.pi, size=(ny, nx)).astype(np.float32).astype(np.float64)
    return dict(nx=nx, ny=ny, modes=modes, w=w, amp=amp, t=t, phi=phi, full=full,
                geom=geom, R=geom.R)


def _ctx(A, h):
    c = A.Context(0)
    c.set_precision(h["full"])
    c.set_basis(h["nx"], h["ny"], modes=h["modes"], R=h["R"],
                amp=torch.tensor(h["amp"], dtype=torch.float32, device="cuda"))
    c.set_spots(h["w"], h["t"])
    return c


def _cu(a):
    return torch.tensor(np.asarray(a), dtype=torch.float32, device="cuda")


def _batch_vs_alone(c, t, ph_b, W_b, ph_1, W_1, E_1, what, n_iter=1):
    """The batch's phase and weights after n_iter iterations against the
    member's own run: the bars follow the step's conditioning for field
    differences of FP32 summation size, n_iter times, never looser than
    1e-4 rad and 1e-5 relative per iteration."""
    t = np.asarray(t, np.float64)
    E1 = E_1.cpu().numpy().astype(np.complex128)
    W1 = W_1.cpu().numpy().astype(np.float64)
    rms = np.sqrt(np.mean(np.abs(E1) ** 2))
    dE = n_iter * FP32_SUM_REL * np.maximum(np.abs(E1), rms)
    wb, sigma = step_bars(E1, dE, W1, t)
    y = (W_1 * torch.tensor(t, dtype=torch.float32, device="cuda")).to(torch.complex64) \
        * E_1 / E_1.abs().clamp_min(1e-30)
    g = c.adjoint(y.to(torch.complex64)).cpu().numpy()
    pe = assert_step_phase(ph_b.cpu().numpy(), ph_1.cpu().numpy(), g, sigma,
                           rel_adj=n_iter * FP32_SUM_REL, what=what + " phase",
                           floor=1e-4 * n_iter)
    we = assert_step_weights(W_b.cpu().numpy(), W1, wb, what=what + " weights",
                             floor=1e-5 * n_iter)
    return pe[0], we[0]


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


@pytest.mark.parametrize("one_launch", [True, False], ids=["one_launch", "per_phase"])
@pytest.mark.parametrize("n_iter", [1, 3])
def test_batch_equals_unbatched(A, batch_case, n_iter, one_launch):
    holos, ctxs = batch_case
    b = A.Batch(ctxs)
    b.set_form(one_launch)
    assert b.info()["one_launch"] == one_launch
    # every member has at most 512 spots: the per-phase iterations after
    # the first run as fused adjoint-and-forward launches
    assert b.info()["fused"]
    ph_b = [_cu(h["phi"]) for h in holos]
    W_b = [torch.ones(h["w"].shape[0], device="cuda") for h in holos]
    b.wgs(ph_b, n_iter, weights=W_b)
    torch.cuda.synchronize()
    for h, c, pb, wb in zip(holos, ctxs, ph_b, W_b):
        ph = _cu(h["phi"])
        _, W, E, _ = c.wgs(ph, n_iter)
        err = _batch_vs_alone(c, h["t"], pb, wb, ph, W, E, "batch vs alone",
                              n_iter)
        _say("holo", h["nx"], h["ny"], h["w"].shape[0], "phase, weights", err)
    b.close()


def test_batch_step_matches_oracle(A, batch_case):
    holos, ctxs = batch_case
    b = A.Batch(ctxs)
    ph_b = [_cu(h["phi"]) for h in holos]
    W_b = [torch.ones(h["w"].shape[0], device="cuda") for h in holos]
    b.wgs(ph_b, 1, weights=W_b)
    for h, c, pb, wb in zip(holos, ctxs, ph_b, W_b):
        basis = oracle.ZernikeBasis(h["modes"])
        N = h["w"].shape[0]
        ref = stepcheck.reference_step(h["phi"], np.ones(N), h["t"], h["amp"],
                                       h["w"], basis, h["geom"])
        # the batch does not return its fields: the member's own forward of
        # the start phase stands for them in the first stage
        E = c.forward(phase=_cu(h["phi"]))
        stepcheck.check_step("batch step %dx%d, %d spots" % (h["nx"], h["ny"], N),
                             pb, wb, E, ref, h["t"])
    b.close()


def test_batch_tuning_table(A, batch_case, tmp_path):
    holos, ctxs = batch_case
    b = A.Batch(ctxs)
    ph = [_cu(h["phi"]) for h in holos]
    path = str(tmp_path / "tune.txt")
    inf = b.tune(ph, table_out=path)
    _say(inf, open(path).read())
    # these members are small: the tuner sets both forms' parameters (range
    # lengths; resident blocks per CU of the one-launch form) and
    # keeps the faster form
    cands = (4, 8, 16, 32, 64, 128) if inf["fused"] else (16, 32, 64, 128, 256, 512)
    assert all(L in cands for L in inf["range_blocks"])
    rows = [l.split() for l in open(path) if not l.startswith("#")]
    assert sum(r[0] == "one_launch" for r in rows) == inf["shapes"]
    assert all(int(r[3]) >= 1 for r in rows if r[0] == "one_launch")
    assert sum(r[0] == "form" for r in rows) == 1
    assert sum(r[0].isdigit() for r in rows) == inf["shapes"]
    b2 = A.Batch(ctxs)
    b2.load_tuning(path)
    i2 = b2.info()
    assert i2["grid"] == inf["grid"]
    assert i2["one_launch"] == inf["one_launch"]
    assert i2["range_blocks"] == inf["range_blocks"]
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


def test_batch64_members(A):
    """The full 64-hologram workload, one batched iteration from the start
    phases.  Every member against its own unbatched iteration (same kernels,
    other partial-sum grouping); the three smallest members (by N * P)
    against the oracle's whole step, in stages; the three largest, whose
    whole step is beyond the oracle's reach in a test (up to 2.0e10
    evaluations per transform), through their unbatched transforms against
    the oracle on 64 sampled spots and 4096 sampled pixels."""
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
    # every member against its unbatched iteration: the two differ by the
    # FP32 summation order of the forward, carried through the step's
    # conditioning (dark spots of the random start phase)
    worst = (0.0, 0.0)
    for h, (d, c) in enumerate(zip(holos, ctxs)):
        p1 = _cu(d["phi0"])
        _, W1, E1, _ = c.wgs(p1, 1)
        err = _batch_vs_alone(c, d["t"], ph[h], W[h], p1, W1, E1,
                              "batch64 member %d vs alone" % h)
        worst = (max(worst[0], err[0]), max(worst[1], err[1]))
    _say("batch vs alone over 64 members: phase %.2e rad, weights %.2e" % worst)
    order = np.argsort([d["w"].shape[0] * d["nx"] * d["ny"] for d in holos])
    rng = np.random.default_rng(64)
    for h in order[:3]:
        d = holos[h]
        geom = oracle.Geometry(d["nx"], d["ny"])
        basis = oracle.ZernikeBasis(d["modes"])
        amp = d["amp"].astype(np.float32).astype(np.float64)
        phi = d["phi0"].astype(np.float32).astype(np.float64)
        t = d["t"].astype(np.float32).astype(np.float64)
        N = d["w"].shape[0]
        # the batch's fields are not returned: the member's own forward of
        # the start phase is the step's first stage
        E = ctxs[h].forward(phase=_cu(phi))
        pix = np.sort(rng.choice(geom.P, size=4096, replace=False))
        ref = stepcheck.reference_step(phi, np.ones(N), t, amp, d["w"], basis,
                                       geom, pixels=pix)
        stepcheck.check_step("batch64 member %d (%d^2, %d spots)" % (h, d["nx"], N),
                             ph[h], W[h], E, ref, t, pixels=pix)
    for h in order[-3:]:
        d = holos[h]
        geom = oracle.Geometry(d["nx"], d["ny"])
        basis = oracle.ZernikeBasis(d["modes"])
        amp = d["amp"].astype(np.float32).astype(np.float64)
        phi = d["phi0"].astype(np.float32).astype(np.float64)
        N = d["w"].shape[0]
        E = ctxs[h].forward(phase=_cu(phi)).cpu().numpy()
        sel = np.sort(rng.choice(N, size=64, replace=False))
        Eref = oracle.forward(amp * np.exp(1j * phi), d["w"], basis, geom, spots=sel)
        _say("batch64 member %d (%d^2, %d spots): forward at 64 spots" % (h, d["nx"], N),
             field_errors(E[sel], Eref))
        assert_fields(E[sel], Eref, what="batch64 member %d forward" % h)
        y = (d["t"] * np.exp(1j * rng.uniform(-np.pi, np.pi, N))).astype(np.complex64)
        g = ctxs[h].adjoint(torch.tensor(y, device="cuda")).cpu().numpy().reshape(-1)
        pix = np.sort(rng.choice(geom.P, size=4096, replace=False))
        gref = oracle.adjoint(y.astype(np.complex128), d["w"], basis, geom, pixels=pix)
        _say("  adjoint at 4096 pixels", field_errors(g[pix], gref))
        assert_fields(g[pix], gref, what="batch64 member %d adjoint" % h)
    b.close()
    for c in ctxs:
        c.close()


def _members(A, holos):
    ctxs = []
    for d in holos:
        c = A.Context(0)
        c.set_basis(d["nx"], d["ny"], modes=d["modes"],
                    amp=torch.tensor(d["amp"], dtype=torch.float32, device="cuda"))
        c.set_spots(d["w"], d["t"])
        ctxs.append(c)
    return ctxs


def test_batch64small_one_launch(A):
    """64 small holograms (256..512 pixels a side, 5..200 spots) in one
    launch per record shape, two iterations: every member against its own
    unbatched run, the three smallest and the three largest (by N * P)
    against the oracle's first step."""
    holos = workloads.make("batch64small")
    ctxs = _members(A, holos)
    b = A.Batch(ctxs)
    b.set_form(True)
    inf = b.info()
    _say(inf)
    assert inf["one_launch"] and sum(inf["grid"]) > 64
    # one iteration against the oracle (three smallest and three largest)
    ph = [_cu(d["phi0"]) for d in holos]
    W = [torch.ones(d["w"].shape[0], device="cuda") for d in holos]
    b.wgs(ph, 1, weights=W)
    torch.cuda.synchronize()
    order = np.argsort([d["w"].shape[0] * d["nx"] * d["ny"] for d in holos])
    rng = np.random.default_rng(6464)
    for h in list(order[:3]) + list(order[-3:]):
        d = holos[h]
        geom = oracle.Geometry(d["nx"], d["ny"])
        basis = oracle.ZernikeBasis(d["modes"])
        amp = d["amp"].astype(np.float32).astype(np.float64)
        phi = d["phi0"].astype(np.float32).astype(np.float64)
        t = d["t"].astype(np.float32).astype(np.float64)
        N = d["w"].shape[0]
        E = ctxs[h].forward(phase=_cu(phi))
        pix = np.sort(rng.choice(geom.P, size=4096, replace=False))
        ref = stepcheck.reference_step(phi, np.ones(N), t, amp, d["w"], basis,
                                       geom, pixels=pix)
        stepcheck.check_step("batch64small member %d (%d^2, %d spots)"
                             % (h, d["nx"], N), ph[h], W[h], E, ref, t,
                             pixels=pix)
    # two more iterations of every member against its own run
    ph2 = [p.clone() for p in ph]
    W2 = [w.clone() for w in W]
    b.wgs(ph, 2, weights=W)
    worst = (0.0, 0.0)
    for h, (d, c) in enumerate(zip(holos, ctxs)):
        p1, w1 = ph2[h], W2[h]
        _, w1, E1, _ = c.wgs(p1, 2, weights=w1)
        err = _batch_vs_alone(c, d["t"], ph[h], W[h], p1, w1, E1,
                              "batch64small member %d vs alone" % h, n_iter=2)
        worst = (max(worst[0], err[0]), max(worst[1], err[1]))
    _say("one launch vs alone over 64 members: phase %.2e rad, weights %.2e" % worst)
    b.close()
    for c in ctxs:
        c.close()


def test_batch64small_deterministic(A):
    """Both batched forms sum their partial rows in a fixed order, so two
    calls from the same start give bitwise the same phases and weights:
    20 iterations of the 64 small holograms in each form (in the one-launch
    form, 20 barriers per hologram whose partial sums every block reads
    from the others)."""
    holos = workloads.make("batch64small")
    ctxs = _members(A, holos)
    b = A.Batch(ctxs)
    for one_launch in (True, False):
        b.set_form(one_launch)
        runs = []
        for _ in range(2):
            ph = [_cu(d["phi0"]) for d in holos]
            W = [torch.ones(d["w"].shape[0], device="cuda") for d in holos]
            b.wgs(ph, 20, weights=W)
            torch.cuda.synchronize()
            runs.append((ph, W))
        (p1, w1), (p2, w2) = runs
        assert all(torch.equal(x, y) for x, y in zip(p1, p2)), one_launch
        assert all(torch.equal(x, y) for x, y in zip(w1, w2)), one_launch
        _say("form %s: two calls bitwise equal" %
             ("one launch" if one_launch else "per phase"))
    b.close()
    for c in ctxs:
        c.close()


def test_batch64small_fused(A):
    """The same 64 holograms in launches per phase, where every iteration
    after the first fuses the adjoint with the next forward: three
    iterations of every member against its own unbatched run."""
    holos = workloads.make("batch64small")
    ctxs = _members(A, holos)
    b = A.Batch(ctxs)
    b.set_form(False)
    inf = b.info()
    assert inf["fused"] and not inf["one_launch"]
    ph = [_cu(d["phi0"]) for d in holos]
    W = [torch.ones(d["w"].shape[0], device="cuda") for d in holos]
    b.wgs(ph, 3, weights=W)
    worst = (0.0, 0.0)
    for h, (d, c) in enumerate(zip(holos, ctxs)):
        p1 = _cu(d["phi0"])
        _, w1, E1, _ = c.wgs(p1, 3)
        err = _batch_vs_alone(c, d["t"], ph[h], W[h], p1, w1, E1,
                              "batch64small member %d fused vs alone" % h,
                              n_iter=3)
        worst = (max(worst[0], err[0]), max(worst[1], err[1]))
    _say("fused vs alone over 64 members: phase %.2e rad, weights %.2e" % worst)
    b.close()
    for c in ctxs:
        c.close()


def test_fused_edges(A):
    """Fused launches at their edges: a member of exactly 512 spots (the
    largest the fused form takes, 40 KB of LDS per block), one spot, 33
    spots (one spot into a second block), last spot blocks of 6, 16 and 24
    spots (the adjoint takes 4, 8 and 12 of a lane's 16 values there), a
    range-reduced record shape and an odd range length loaded from a
    table; three iterations of every member against its own run."""
    specs = [
        (160, 96, 512, [1, 2, 3, 4, 5, 7, 12], 0.4, 1.0, False, None),
        (64, 48, 1, [1, 2, 4], 0.3, 1.0, False, None),
        (96, 80, 33, [1, 2, 3, 4, 5, 7, 12], 0.6, 1.0, False, None),
        (48, 40, 70, [1, 2, 4, 7], 0.7, 9.0, False, None),
        (64, 64, 48, [1, 2, 4], 0.5, 1.0, False, None),
        (80, 64, 88, [1, 2, 3, 4, 5, 7, 12], 0.5, 1.0, False, None),
    ]
    holos = [_holo(s, 900 + i) for i, s in enumerate(specs)]
    ctxs = [_ctx(A, h) for h in holos]
    assert any(c.info()["range_reduce"] for c in ctxs)
    b = A.Batch(ctxs)
    b.set_form(False)
    assert b.info()["fused"]
    import tempfile
    with tempfile.TemporaryDirectory() as tmp:
        path = os.path.join(tmp, "odd.txt")
        with open(path, "w") as f:
            for inf in (c.info() for c in ctxs):
                f.write("%d %d 7 0.0\n" % (inf["groups"], inf["range_reduce"]))
        b.load_tuning(path)
    assert all(L == 8 for L in b.info()["range_blocks"])  # made even
    ph_b = [_cu(h["phi"]) for h in holos]
    W_b = [torch.ones(h["w"].shape[0], device="cuda") for h in holos]
    b.wgs(ph_b, 3, weights=W_b)
    # the same members in the one-launch form, which runs the same rows
    b.set_form(True)
    ph_o = [_cu(h["phi"]) for h in holos]
    W_o = [torch.ones(h["w"].shape[0], device="cuda") for h in holos]
    b.wgs(ph_o, 3, weights=W_o)
    torch.cuda.synchronize()
    for h, c, pb, wb, po, wo in zip(holos, ctxs, ph_b, W_b, ph_o, W_o):
        ph = _cu(h["phi"])
        _, W, E, _ = c.wgs(ph, 3)
        err = _batch_vs_alone(c, h["t"], pb, wb, ph, W, E, "fused edge", 3)
        _say("  %dx%d, %d spots: phase, weights" % (h["nx"], h["ny"], h["w"].shape[0]), err)
        err = _batch_vs_alone(c, h["t"], po, wo, ph, W, E, "one-launch edge", 3)
        _say("    one launch: phase, weights", err)
    b.close()
    for c in ctxs:
        c.close()


def test_batch64_uses_phase_launches(A):
    """Members with more spots than the one-launch form holds run as one
    launch per phase (the batch64 test covers their results)."""
    d = max(workloads.make("batch64"), key=lambda x: x["w"].shape[0])
    ctxs = _members(A, [d])
    b = A.Batch(ctxs)
    assert d["w"].shape[0] > 512 and not b.info()["one_launch"]
    assert not b.info()["fused"]
    with pytest.raises(A.AshError):
        b.set_form(True)
    b.close()
    for c in ctxs:
        c.close()
