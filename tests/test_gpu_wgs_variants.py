"""GPU parity of the weighted-GS variants: phase-fixed WGS and experimental
feedback (ash_wgs_iterate's fix_phase_after, ash_wgs_feedback), one step at a
time from the oracle's state (FP32 and FP64 trajectories drift apart, so
whole runs are not compared)."""

import sys

import numpy as np
import pytest

import oracle
import stepcheck
import workloads
from tolerance import assert_fields, assert_phase, field_errors, STEP_PHASE_MASK

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


def _setup(A):
    d = workloads.plain256()
    geom = oracle.Geometry(d["nx"], d["ny"])
    basis = oracle.ZernikeBasis(d["modes"])
    amp = d["amp"].astype(np.float32).astype(np.float64)
    phi0 = d["phi0"].astype(np.float32).astype(np.float64)
    c = A.Context(0)
    c.set_basis(d["nx"], d["ny"], modes=d["modes"],
                amp=torch.tensor(d["amp"], dtype=torch.float32, device="cuda"))
    c.set_spots(d["w"], d["t"])
    return d, geom, basis, amp, phi0, c


def _cuda(x):
    return torch.tensor(np.asarray(x), dtype=torch.float32, device="cuda")


def test_phase_fixed_step_matches_oracle(A):
    d, geom, basis, amp, phi0, c = _setup(A)
    t = d["t"]
    # oracle: 3 free iterations, the phases of iteration 2 fixed afterwards
    _, _, _, _, kept = oracle.wgs_run(phi0, t, amp, d["w"], basis, geom, 5,
                                      keep=(2, 3, 4), fix_phase_after=3)
    phi2, W2 = kept[2]
    _, _, E2, _ = oracle.wgs_step(phi2, W2, t, amp, d["w"], basis, geom)
    psi = np.angle(E2)
    for it in (3, 4):
        phi_i, W_i = kept[it]
        phi_i = phi_i.astype(np.float32).astype(np.float64)
        W_i = W_i.astype(np.float32).astype(np.float64)
        # the GPU stores its own arg E of iteration 2 from the oracle's state
        ph = _cuda(phi2)
        _, _, Eg2, _ = c.wgs(ph, 1, weights=_cuda(W2), fix_phase_after=1)
        _say("  stored fields", field_errors(Eg2.cpu().numpy(), E2))
        assert_fields(Eg2.cpu().numpy(), E2, what="fields of the stored step")
        ph = _cuda(phi_i)
        Wt = _cuda(W_i)
        _, Wg, Eg, _ = c.wgs(ph, 1, weights=Wt, fix_phase_after=-1)
        ref_phi, ref_W, ref_E, _ = oracle.wgs_step(phi_i, W_i, t, amp, d["w"],
                                                   basis, geom, fixed_phase=psi)
        np.testing.assert_allclose(Wg.cpu().numpy(), ref_W, rtol=2e-4)
        y, _ = oracle.wgs_farfield(ref_E, W_i, t, fixed_phase=psi)
        gref = oracle.adjoint(y, d["w"], basis, geom)
        _say("  phase @%d" % it, assert_phase(ph.cpu().numpy(), ref_phi, gref,
                                              mask=STEP_PHASE_MASK,
                                              what="phase-fixed step %d" % it))
    c.close()


def test_storing_step_equals_free_step_and_fixed_needs_store(A):
    d, geom, basis, amp, phi0, c = _setup(A)
    W = _cuda(np.ones(d["w"].shape[0]))
    a = _cuda(phi0)
    b = _cuda(phi0)
    Wa, Wb = W.clone(), W.clone()
    from paper_2505_08777_amd import AshError
    with pytest.raises(AshError):
        c.wgs(a.clone(), 1, weights=Wa.clone(), fix_phase_after=-1)
    c.wgs(a, 2, weights=Wa, fix_phase_after=0)
    c.wgs(b, 2, weights=Wb, fix_phase_after=2)
    assert torch.equal(a, b) and torch.equal(Wa, Wb)
    # set_spots forgets the stored phases
    c.set_spots(d["w"], d["t"])
    with pytest.raises(AshError):
        c.wgs(a, 1, weights=Wa, fix_phase_after=-1)
    c.close()


def test_feedback_step_matches_oracle(A):
    """Weights driven by 'measured' amplitudes: the model's |E| times fixed
    per-spot factors (a system whose spots are brighter or dimmer than
    modelled), from the oracle's state at iterations 0 and 5."""
    d, geom, basis, amp, phi0, c = _setup(A)
    t = d["t"]
    N = d["w"].shape[0]
    rng = np.random.default_rng(77)
    gain = rng.uniform(0.7, 1.3, size=N)
    gain[3] = 0.0                                   # a dark spot
    _, _, _, _, kept = oracle.wgs_run(phi0, t, amp, d["w"], basis, geom, 6,
                                      keep=(0, 5))
    for it in (0, 5):
        phi_i, W_i = kept[it]
        phi_i = phi_i.astype(np.float32).astype(np.float64)
        W_i = W_i.astype(np.float32).astype(np.float64)
        E_i = oracle.forward(amp * np.exp(1j * phi_i), d["w"], basis, geom)
        meas = (gain * np.abs(E_i)).astype(np.float32).astype(np.float64)
        ph = _cuda(phi_i)
        Wt = _cuda(W_i)
        _, Wg, Eg, st = c.wgs_feedback(ph, _cuda(meas), weights=Wt)
        ref_phi, ref_W, ref_E, ref_st = oracle.wgs_step(
            phi_i, W_i, t, amp, d["w"], basis, geom, measured=meas)
        _say("  fields @%d" % it, field_errors(Eg.cpu().numpy(), ref_E))
        assert_fields(Eg.cpu().numpy(), ref_E, what="feedback fields")
        np.testing.assert_allclose(Wg.cpu().numpy(), ref_W, rtol=2e-4)
        y, _ = oracle.wgs_farfield(ref_E, W_i, t, measured=meas)
        gref = oracle.adjoint(y, d["w"], basis, geom)
        _say("  phase @%d" % it, assert_phase(ph.cpu().numpy(), ref_phi, gref,
                                              mask=STEP_PHASE_MASK,
                                              what="feedback step %d" % it))
        np.testing.assert_allclose(st.cpu().numpy(), ref_st, rtol=1e-3, atol=1e-3)
    c.close()


def test_resume_is_bitwise(A):
    """Checkpoint and resume: 8 iterations in one call equal 3 + 5 in two
    calls, and a phase-fixed run resumed in a fresh context from (phase,
    weights, stored farfield phases) equals the uninterrupted run, bitwise
    (the reductions have a fixed order)."""
    d, geom, basis, amp, phi0, c = _setup(A)
    N = d["w"].shape[0]
    a = _cuda(phi0)
    Wa = _cuda(np.ones(N))
    c.wgs(a, 8, weights=Wa)
    b = _cuda(phi0)
    Wb = _cuda(np.ones(N))
    c.wgs(b, 3, weights=Wb)
    c.wgs(b, 5, weights=Wb)
    assert torch.equal(a, b) and torch.equal(Wa, Wb)
    # phase fixed after 3 iterations, 8 in all
    p1 = _cuda(phi0)
    W1 = _cuda(np.ones(N))
    c.wgs(p1, 8, weights=W1, fix_phase_after=3)
    p2 = _cuda(phi0)
    W2 = _cuda(np.ones(N))
    c.wgs(p2, 4, weights=W2, fix_phase_after=3)
    psi = c.fixed_phases().clone()           # checkpoint
    c2 = A.Context(0)
    c2.set_basis(d["nx"], d["ny"], modes=d["modes"],
                 amp=torch.tensor(d["amp"], dtype=torch.float32, device="cuda"))
    c2.set_spots(d["w"], d["t"])
    c2.set_fixed_phases(psi)                  # resume elsewhere
    c2.wgs(p2, 4, weights=W2, fix_phase_after=-1)
    assert torch.equal(p1, p2) and torch.equal(W1, W2)
    assert torch.equal(c2.fixed_phases(), c.fixed_phases())
    c2.close()
    c.close()


@pytest.mark.parametrize("start", ["random", "iteration3"])
def test_many_spot_update_paths_match_oracle(A, start):
    """More spots than the update block has threads (2500 > 1024, so fields
    and weights go through memory): a free step, a phase-fixed step and a
    feedback step, each against the oracle's step from the same state,
    judged in stages (fields, then weights and phases at the bars the field
    errors imply through the step).  From the random start phase some spots
    are nearly dark and the step is ill-conditioned in them; from the
    oracle's state after three iterations it is not."""
    nx, ny, N = 96, 64, 2500
    modes = [1, 2, 3, 4, 5]
    rng = np.random.default_rng(2500)
    geom = oracle.Geometry(nx, ny)
    basis = oracle.ZernikeBasis(modes)
    w = rng.normal(0, 0.4, size=(N, len(modes)))
    w[:, 0] = np.pi * rng.uniform(-ny / 2, ny / 2, N) * geom.R / ny
    w[:, 1] = np.pi * rng.uniform(-nx / 2, nx / 2, N) * geom.R / nx
    t = rng.uniform(0.5, 1.0, N).astype(np.float32).astype(np.float64)
    amp = rng.uniform(0.2, 1.0, (ny, nx)).astype(np.float32).astype(np.float64)
    phi0 = rng.uniform(-np.pi, np.pi, (ny, nx)).astype(np.float32).astype(np.float64)
    if start == "random":
        phi, W0 = phi0, np.ones(N)
    else:
        _, _, _, _, kept = oracle.wgs_run(phi0, t, amp, w, basis, geom, 4,
                                          keep=(3,))
        phi = kept[3][0].astype(np.float32).astype(np.float64)
        W0 = kept[3][1].astype(np.float32).astype(np.float64)
    c = A.Context(0)
    c.set_basis(nx, ny, modes=modes, amp=_cuda(amp))
    c.set_spots(w, t)
    _say("start", start)

    # free step, storing its farfield phases
    ph = _cuda(phi)
    _, Wg, Eg, _ = c.wgs(ph, 1, weights=_cuda(W0), fix_phase_after=1)
    ref = stepcheck.reference_step(phi, W0, t, amp, w, basis, geom)
    free = stepcheck.check_step("free", ph, Wg, Eg, ref, t)
    E_free = ref[0]
    # the stored phases used from the same start: they are the GPU's own
    # free-step phases, against the oracle's arg E of that step
    ph = _cuda(phi)
    _, Wg, Eg, _ = c.wgs(ph, 1, weights=_cuda(W0), fix_phase_after=-1)
    ref = stepcheck.reference_step(phi, W0, t, amp, w, basis, geom,
                                   fixed_phase=np.angle(E_free))
    stepcheck.check_step("fixed", ph, Wg, Eg, ref, t,
                         dpsi=free["abs_dE"] / np.abs(E_free))
    # feedback: measured amplitudes replace |E| in the weight update
    meas = (rng.uniform(0.7, 1.3, N) * np.abs(E_free)).astype(np.float32)
    meas = meas.astype(np.float64)
    ph = _cuda(phi)
    _, Wg, Eg, _ = c.wgs_feedback(ph, _cuda(meas), weights=_cuda(W0))
    ref = stepcheck.reference_step(phi, W0, t, amp, w, basis, geom,
                                   measured=meas)
    stepcheck.check_step("feedback", ph, Wg, Eg, ref, t,
                         weights_from_fields=False)
    c.close()
