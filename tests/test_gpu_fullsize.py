"""Full-size parity in the benchmarked configuration.

The 1024 x 1024 / 400-spot and 1920 x 1200 / 2000-spot WGS workloads are
built exactly as the benchmark builds them (default precision, the same
launch plan).  Each forward output depends on one spot and each adjoint
output on one pixel, so sampled outputs from the FP64 oracle are exact
references: 64 spots over all pixels, and 4096 pixels over all spots.  At
1024 x 1024 one whole WGS step is also checked on the sampled pixels (the
oracle's forward there runs over every spot), from the random start and
from the oracle's own states at iterations 1, 10 and 99; at 1920 x 1200
one step from the random start, the oracle's forward over every spot.
"""

import json
import os
import sys

import numpy as np
import pytest

import oracle
import stepcheck
import workloads
from tolerance import (assert_fields, assert_phase, field_errors,
                       STEP_PHASE_MASK)

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def A():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2505_08777_amd as A
    return A


def _setup(A, name):
    d = workloads.make(name)
    c = A.Context(0)
    c.set_basis(d["nx"], d["ny"], modes=d["modes"],
                amp=torch.tensor(d["amp"], dtype=torch.float32, device="cuda"))
    c.set_spots(d["w"], d["t"])
    geom = oracle.Geometry(d["nx"], d["ny"])
    basis = oracle.ZernikeBasis(d["modes"])
    amp = d["amp"].astype(np.float32).astype(np.float64)
    phi = d["phi0"].astype(np.float32).astype(np.float64)
    return d, c, geom, basis, amp, phi


@pytest.mark.parametrize("name", ["field1024", "volume1920"])
def test_fullsize_sampled_transforms(A, name):
    d, c, geom, basis, amp, phi = _setup(A, name)
    N = d["w"].shape[0]
    _say("case", name, c.info())
    rng = np.random.default_rng(7 + N)
    ph = torch.tensor(phi, dtype=torch.float32, device="cuda")
    E = c.forward(phase=ph).cpu().numpy()
    sel = np.sort(rng.choice(N, size=64, replace=False))
    Eref = oracle.forward(amp * np.exp(1j * phi), d["w"], basis, geom,
                          spots=sel)
    _say("  forward (64 spots)", field_errors(E[sel], Eref))
    assert_fields(E[sel], Eref, what="forward at sampled spots")
    # a farfield like the loop's: unit-magnitude spot phases times targets
    y = (d["t"] * np.exp(1j * rng.uniform(-np.pi, np.pi, N))).astype(np.complex64)
    g, phg = c.adjoint(torch.tensor(y, device="cuda"), field=True, phase=True)
    g = g.cpu().numpy().reshape(-1)
    phg = phg.cpu().numpy().reshape(-1)
    pix = np.sort(rng.choice(geom.P, size=4096, replace=False))
    gref = oracle.adjoint(y.astype(np.complex128), d["w"], basis, geom,
                          pixels=pix)
    _say("  adjoint (4096 pixels)", field_errors(g[pix], gref))
    assert_fields(g[pix], gref, what="adjoint at sampled pixels")
    assert_phase(phg[pix], np.angle(gref), gref, what="adjoint phase")
    c.close()


def _golden_state(k):
    with open(os.path.join(GOLDEN, "field1024_states.json")) as fh:
        st = json.load(fh)["states"][str(k)]
    return (np.asarray(st["y_re"]) + 1j * np.asarray(st["y_im"]),
            np.asarray(st["W"]))


@pytest.mark.parametrize("k", [0, 1, 10, 99])
def test_fullsize_wgs_step_field1024(A, k):
    """One WGS step at 1024 x 1024 with 400 spots from the state entering
    iteration k of the oracle's own run (k = 0: the workload's random start
    phase, unit weights; later states from tests/golden/field1024_states.json,
    written by the oracle), against the oracle's step from the same state:
    all fields, all weights, phases at 4096 sampled pixels."""
    d, c, geom, basis, amp, phi = _setup(A, "field1024")
    N = d["w"].shape[0]
    t = d["t"].astype(np.float32).astype(np.float64)
    W = np.ones(N)
    if k > 0:
        y_prev, W = _golden_state(k)
        phi = np.angle(oracle.adjoint(y_prev, d["w"], basis, geom))
        phi = phi.astype(np.float32).astype(np.float64)
        W = W.astype(np.float32).astype(np.float64)
    _say("state entering iteration", k)
    ph = torch.tensor(phi, dtype=torch.float32, device="cuda")
    Wt = torch.tensor(W, dtype=torch.float32, device="cuda")
    _, Wg, Eg, _ = c.wgs(ph, 1, weights=Wt)
    rng = np.random.default_rng(1024 + k)
    pix = np.sort(rng.choice(geom.P, size=4096, replace=False))
    ref = stepcheck.reference_step(phi, W, t, amp, d["w"], basis, geom,
                                   pixels=pix)
    stepcheck.check_step("field1024 step %d" % k, ph, Wg, Eg, ref, t,
                         pixels=pix)
    c.close()


def test_fullsize_wgs_step_volume1920(A):
    """One WGS step at 1920 x 1200 with 2000 spots from the workload's random
    start phase: the oracle's forward over every spot and pixel (4.6 G
    evaluations), its weight update, and its adjoint at 4096 sampled
    pixels, against the GPU's step in the benchmarked set-up."""
    d, c, geom, basis, amp, phi = _setup(A, "volume1920")
    N = d["w"].shape[0]
    t = d["t"].astype(np.float32).astype(np.float64)
    _say("case volume1920 step 0", c.info())
    ph = torch.tensor(phi, dtype=torch.float32, device="cuda")
    Wt = torch.ones(N, dtype=torch.float32, device="cuda")
    _, Wg, Eg, _ = c.wgs(ph, 1, weights=Wt)
    rng = np.random.default_rng(1920)
    pix = np.sort(rng.choice(geom.P, size=4096, replace=False))
    ref = stepcheck.reference_step(phi, np.ones(N), t, amp, d["w"], basis,
                                   geom, pixels=pix)
    stepcheck.check_step("volume1920 step 0", ph, Wg, Eg, ref, t, pixels=pix)
    c.close()
