"""The oracle's pins catch plausible mistakes.

Each case plants one mistake in the FP64 oracle (on the CPU, through
monkeypatch, so the oracle's files stay as they are) and runs the pins of
``test_oracle_pins.py``; at least one pin must fail.  The mistakes are the
kinds a reader would look for: a flipped sign, transposed or shifted
coordinates, a wrong normalisation, a dropped term, a non-conjugate adjoint,
a wrong weight exponent, a dropped TV factor, a wrong gradient sign.
"""

import math

import numpy as np
import pytest

import oracle
import oracle.grad as ograd
import oracle.principal as oprincipal
import oracle.quality as oquality
import oracle.transform as otransform
import oracle.wgs as owgs
import oracle.zernike as ozernike
import test_oracle_pins as pins
import test_oracle_principal as ppins

# every pin, with the parameters it is collected with
PIN_CALLS = [
    ("test_paper_index_facts", {}),
    ("test_ansi_roundtrip_and_noll_map", {}),
    ("test_zernike_textbook_cartesian", {}),
    ("test_zernike_jacobi_route", {}),
    ("test_zernike_orthonormal_quadrature", {}),
    ("test_monomial_basis_matches_direct", {}),
    ("test_forward_integer_bins_equal_fft", {"nx": 24, "ny": 16}),
    ("test_forward_odd_sizes_general_phase", {}),
    ("test_adjoint_integer_bins_equal_ifft", {}),
    ("test_dirichlet_off_grid", {}),
    ("test_quadratic_gauss_sum", {"n": 64}),
    ("test_conjugate_hologram_textbook_phase", {}),
    ("test_dot_product_adjoint", {}),
    ("test_piston_linearity_aliasing_subsets", {}),
    ("test_bruteforce_mpmath_8x8", {}),
    ("test_one_spot_wgs_reaches_sum_amp", {}),
    ("test_wgs_equals_fft_wgs_at_integer_bins", {"power": 1.0}),
    ("test_wgs_stats_definitions", {}),
    ("test_feedback_weight_update_closed_forms", {}),
    ("test_phase_fixed_projection_against_fft", {}),
    ("test_fd_update_equals_full_recompute_and_analytic", {}),
    ("test_adam_first_step_closed_form", {}),
    ("test_adam_run_descends_and_uses_loss_grad", {}),
    ("test_moments_are_central_differences_of_the_fields", {}),
    ("test_piston_moment_is_the_field_and_tilt_moment_closed_form", {}),
    ("test_window_strehl_of_a_perfect_spot_closed_form",
     {"step": 0.5, "win": 7}),
    ("test_window_strehl_invariances_and_layout", {}),
] + [(ppins, name, {}) for name in (
    "test_known_spectrum_and_eckart_young", "test_rank_k_matrix_is_exact",
    "test_full_rank_keeps_phases_and_k0_keeps_linear_part",
    "test_phase_change_within_cauchy_schwarz_bound",
    "test_rank_one_direction")]


def _failing_pins():
    failed = []
    for call in PIN_CALLS:
        mod, name, kw = call if len(call) == 3 else (pins,) + call
        try:
            getattr(mod, name)(**kw)
        except pytest.skip.Exception:
            continue
        except Exception:  # an assertion or an error both count
            failed.append(name)
    return failed


def _patch_both(mp, module, name, value):
    """Replace `name` in its defining module, the package and the pins."""
    mp.setattr(module, name, value)
    if hasattr(oracle, name):
        mp.setattr(oracle, name, value)
    if hasattr(pins, name):
        mp.setattr(pins, name, value)


def _kernel_sign(mp):
    kp = otransform.kernel_phase
    _patch_both(mp, otransform, "kernel_phase",
                lambda w, basis, geom, idx: -kp(w, basis, geom, idx))


def _transposed_coords(mp):
    orig = otransform.Geometry.coords

    def coords(self, flat_idx):
        xh, yh = orig(self, flat_idx)
        return yh, xh
    mp.setattr(otransform.Geometry, "coords", coords)


def _shifted_coords(mp):
    orig = otransform.Geometry.coords

    def coords(self, flat_idx):
        xh, yh = orig(self, flat_idx)
        return xh + 1.0 / self.R, yh
    mp.setattr(otransform.Geometry, "coords", coords)


def _zernike_norm(mp):
    zn = ozernike.zernike_nm

    def wrong(n, m, x, y):
        z = zn(n, m, x, y)
        return z / math.sqrt(2.0) if m != 0 else z
    _patch_both(mp, ozernike, "zernike_nm", wrong)


def _radial_dropped_term(mp):
    def radial(n, am, rho):
        out = np.zeros_like(rho, dtype=np.float64)
        for s in range((n - am) // 2):          # the last term is dropped
            c = ((-1) ** s * math.factorial(n - s)
                 / (math.factorial(s) * math.factorial((n + am) // 2 - s)
                    * math.factorial((n - am) // 2 - s)))
            out = out + c * rho ** (n - 2 * s)
        return out if (n - am) // 2 > 0 else out + rho ** n
    mp.setattr(ozernike, "radial", radial)


def _adjoint_not_conjugate(mp):
    adj = otransform.adjoint

    def wrong(y, *a, **k):
        return np.conj(adj(np.conj(np.asarray(y)), *a, **k))
    _patch_both(mp, otransform, "adjoint", wrong)
    mp.setattr(owgs, "adjoint", wrong)
    mp.setattr(ograd, "adjoint", wrong)


def _weight_exponent(mp):
    ff = owgs.wgs_farfield

    def wrong(E, weights, t, power=1.0, measured=None, fixed_phase=None):
        return ff(E, weights, t, -power, measured, fixed_phase)
    _patch_both(mp, owgs, "wgs_farfield", wrong)


def _tv_factor(mp):
    tg = ograd.tv_grad
    _patch_both(mp, ograd, "tv_grad",
                lambda phi, eps=1e-3: tg(phi, eps) * np.asarray(phi).size)


def _grad_sign(mp):
    lg = ograd.loss_grad

    def wrong(*a, **k):
        g, L, E = lg(*a, **k)
        return -g, L, E
    _patch_both(mp, ograd, "loss_grad", wrong)


def _moment_conjugate(mp):
    fm = ograd.forward_moments
    _patch_both(mp, ograd, "forward_moments",
                lambda *a, **k: np.conj(fm(*a, **k)))


def _strehl_amplitudes(mp):
    def wrong(E, N, win):
        a = np.abs(np.asarray(E, dtype=np.complex128)).reshape(N, win * win)
        tot = a.sum(axis=1)
        return np.where(tot > 0, a.max(axis=1) / np.where(tot > 0, tot, 1.0),
                        0.0)
    _patch_both(mp, oquality, "window_strehl", wrong)


def _window_axes_swapped(mp):
    wc = oquality.window_coefficients
    _patch_both(mp, oquality, "window_coefficients",
                lambda w, ix, iy, dwx, dwy, win: wc(w, iy, ix, dwy, dwx, win))


def _spread_sample_std(mp):
    ws = owgs.wgs_stats

    def wrong(E, t, amp):
        st = np.array(ws(E, t, amp), dtype=np.float64)
        I = np.abs(np.asarray(E)) ** 2 / np.asarray(t, dtype=np.float64) ** 2
        mu = np.mean(I)
        st[2] = np.std(I, ddof=1) / mu if mu > 0 else 0.0
        return st
    _patch_both(mp, owgs, "wgs_stats", wrong)


def _principal_trailing(mp):
    def wrong(w, basis, K):
        w = np.asarray(w, dtype=np.float64)
        lin = oprincipal.linear_modes(basis)
        keep, rot = np.flatnonzero(lin), np.flatnonzero(~lin)
        WR = w[:, rot]
        _, sv, Vt = np.linalg.svd(WR, full_matrices=True)
        sigma = np.zeros(rot.size)
        sigma[:sv.size] = sv
        VK = Vt[::-1][:K].T                  # the trailing singular vectors
        wK = np.concatenate([w[:, keep], WR @ VK], axis=1)
        return wK, oprincipal.RotatedBasis(basis, keep, rot, VK), sigma
    _patch_both(mp, oprincipal, "principal_modes", wrong)


MUTATIONS = {
    "kernel phase sign": _kernel_sign,
    "transposed pupil coordinates": _transposed_coords,
    "pupil coordinates shifted by one pixel": _shifted_coords,
    "Zernike normalisation of m != 0": _zernike_norm,
    "last radial term dropped": _radial_dropped_term,
    "adjoint not the conjugate transpose": _adjoint_not_conjugate,
    "WGS weight exponent sign": _weight_exponent,
    "TV gradient missing its 1/P": _tv_factor,
    "loss gradient sign": _grad_sign,
    "moments conjugated": _moment_conjugate,
    "windowed Strehl of amplitudes, not intensities": _strehl_amplitudes,
    "window offsets on swapped axes": _window_axes_swapped,
    "principal modes from the trailing singular vectors": _principal_trailing,
    "intensity spread with the sample standard deviation": _spread_sample_std,
}


def test_pins_pass_unmutated():
    assert _failing_pins() == []


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_a_pin_catches(name, monkeypatch):
    with monkeypatch.context() as mp:
        MUTATIONS[name](mp)
        failed = _failing_pins()
    print(name, "caught by", failed)
    assert failed, "no pin catches: " + name
