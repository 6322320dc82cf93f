"""Python binding of libash: argument marshalling around the C ABI.

Every transform, reduction and update runs in the library's HIP kernels;
torch supplies device memory (tensors) and the stream.  Pixel arrays are
[ny, nx] float32 (phase, amplitude) or complex64 (fields); spot arrays are
[N] complex64 (fields) or float32 (targets, weights).
"""

import ctypes

import numpy as np
import torch

from ._lib import (lib, check, AshError, WgsParams, AdamParams, Info,
                   BatchInfo, PRECISION_AUTO, PRECISION_FULL)
from .basis import zernike_table


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _dev(t, dtype, shape, name, device):
    if t.device.type != "cuda" or t.device.index != device:
        raise ValueError("%s must be on cuda:%d" % (name, device))
    if t.dtype != dtype:
        raise TypeError("%s must be %s, got %s" % (name, dtype, t.dtype))
    if tuple(t.shape) != tuple(shape):
        raise ValueError("%s must have shape %s, got %s"
                         % (name, tuple(shape), tuple(t.shape)))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    return t


class Context:
    """One library context on one device, enqueueing on torch's stream."""

    def __init__(self, device=0):
        self.device = int(device)
        self._h = ctypes.c_void_p()
        rc = lib.ash_create(ctypes.byref(self._h), self.device, None)
        if rc != 0:
            raise AshError(rc, "ash_create", lib.ash_last_error(None).decode())
        self.nx = self.ny = self.N = self.D = None
        self.cx = self.cy = self.R = None
        self.modes = None
        self.target = None
        # bumped by every set_basis / set_spots (generation) and by every
        # set_basis (basis_generation): a backward pass checks that the basis
        # and spots its forward used are still the context's
        self.generation = 0
        self.basis_generation = 0

    # -- lifetime ---------------------------------------------------------
    def close(self):
        if self._h:
            lib.ash_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def _stream(self):
        s = torch.cuda.current_stream(self.device).cuda_stream
        check(lib.ash_set_stream(self._h, ctypes.c_void_p(s)), "ash_set_stream")

    PROFILE_CATEGORIES = ("forward", "adjoint", "reduce", "field")

    def profile(self, enable=True, categories=None, stride=1):
        """Bracket the kernels of the given categories (default all) with
        HIP events, one launch in every `stride` of each category; see
        profile_read."""
        check(lib.ash_profile_stride(self._h, int(stride)),
              "ash_profile_stride", self._h)
        mask = 0
        if enable:
            cats = self.PROFILE_CATEGORIES if categories is None else categories
            for k in cats:
                mask |= 1 << self.PROFILE_CATEGORIES.index(k)
        check(lib.ash_profile_enable(self._h, mask), "ash_profile_enable",
              self._h)

    def profile_read(self):
        """{category: (total ms, launches)} since the last read; syncs."""
        ms = np.zeros(4, dtype=np.float64)
        n = np.zeros(4, dtype=np.int64)
        check(lib.ash_profile_read(self._h, ms.ctypes.data, n.ctypes.data),
              "ash_profile_read", self._h)
        return {k: (float(ms[i]), int(n[i]))
                for i, k in enumerate(self.PROFILE_CATEGORIES)}

    def set_precision(self, full=False):
        """3 bf16 pieces for every remainder term (full) or the automatic
        choice; takes effect at the next set_spots."""
        check(lib.ash_set_precision(self._h, PRECISION_FULL if full
                                    else PRECISION_AUTO),
              "ash_set_precision", self._h)

    def info(self):
        out = Info()
        check(lib.ash_get_info(self._h, ctypes.byref(out)), "ash_get_info",
              self._h)
        return {f: getattr(out, f) for f, _ in Info._fields_}

    def sync(self):
        check(lib.ash_sync(self._h), "ash_sync", self._h)

    # -- set-up -----------------------------------------------------------
    def set_basis(self, nx, ny, modes=None, mono_pow=None, mono_coef=None,
                  amp=None, cx=None, cy=None, R=None):
        """Zernike modes (ANSI list) or an explicit monomial table."""
        if modes is not None:
            mono_pow, mono_coef = zernike_table(modes)
            self.modes = list(modes)
        mono_pow = np.ascontiguousarray(mono_pow, dtype=np.int32)
        mono_coef = np.ascontiguousarray(mono_coef, dtype=np.float64)
        cx = nx / 2.0 if cx is None else cx
        cy = ny / 2.0 if cy is None else cy
        R = min(nx, ny) / 2.0 if R is None else R
        if amp is not None:
            amp = _dev(amp, torch.float32, (ny, nx), "amp", self.device)
        self._stream()
        check(lib.ash_set_basis(self._h, int(nx), int(ny), float(cx),
                                float(cy), float(R), mono_coef.shape[0],
                                mono_pow.shape[0], mono_pow.ctypes.data,
                                mono_coef.ctypes.data, _ptr(amp)),
              "ash_set_basis", self._h)
        self.nx, self.ny, self.D = int(nx), int(ny), mono_coef.shape[0]
        self.cx, self.cy, self.R = float(cx), float(cy), float(R)
        self.N = None
        self.target = None
        self.generation += 1
        self.basis_generation += 1

    def set_spots(self, w, target=None):
        w = np.ascontiguousarray(w, dtype=np.float64)
        if w.ndim != 2 or w.shape[1] != self.D:
            raise ValueError("w must be [N, %s]" % self.D)
        t = None
        if target is not None:
            t = np.ascontiguousarray(target, dtype=np.float32)
            if t.shape != (w.shape[0],):
                raise ValueError("target must be [N]")
        self._stream()
        check(lib.ash_set_spots(self._h, w.shape[0], w.ctypes.data,
                                t.ctypes.data if t is not None else None),
              "ash_set_spots", self._h)
        self.N = w.shape[0]
        self.target = t
        self.generation += 1

    # -- transforms ---------------------------------------------------------
    def forward(self, phase=None, field=None, out=None):
        """E_n = sum_x f(x) exp(-i theta_n(x)); f = A exp(i phase) or field."""
        if (phase is None) == (field is None):
            raise ValueError("give exactly one of phase, field")
        P = (self.ny, self.nx)
        if phase is not None:
            _dev(phase, torch.float32, P, "phase", self.device)
        else:
            _dev(field, torch.complex64, P, "field", self.device)
        if out is None:
            out = torch.empty(self.N, dtype=torch.complex64,
                              device="cuda:%d" % self.device)
        _dev(out, torch.complex64, (self.N,), "out", self.device)
        self._stream()
        check(lib.ash_forward(self._h, _ptr(phase), _ptr(field), _ptr(out)),
              "ash_forward", self._h)
        return out

    def adjoint(self, y, field=True, phase=False):
        """g(x) = sum_n y_n exp(+i theta_n(x)); returns g and/or arg g."""
        _dev(y, torch.complex64, (self.N,), "y", self.device)
        if not (field or phase):
            raise ValueError("request at least one output")
        dev = "cuda:%d" % self.device
        g = torch.empty((self.ny, self.nx), dtype=torch.complex64,
                        device=dev) if field else None
        ph = torch.empty((self.ny, self.nx), dtype=torch.float32,
                         device=dev) if phase else None
        self._stream()
        check(lib.ash_adjoint(self._h, _ptr(y), _ptr(g), _ptr(ph)),
              "ash_adjoint", self._h)
        if field and phase:
            return g, ph
        return g if field else ph

    def wgs(self, phase, n_iter, weights=None, power=1.0, want_E=True,
            want_stats=True, fix_phase_after=0):
        """n_iter weighted-GS iterations; phase is updated in place.
        fix_phase_after: 0 free farfield phases; n > 0 fixed after the
        first n iterations; < 0 fixed at the phases stored earlier.

        Returns (phase, weights, E_last, stats[n_iter, 4])."""
        _dev(phase, torch.float32, (self.ny, self.nx), "phase", self.device)
        dev = "cuda:%d" % self.device
        if weights is None:
            weights = torch.ones(self.N, dtype=torch.float32, device=dev)
        _dev(weights, torch.float32, (self.N,), "weights", self.device)
        E = torch.empty(self.N, dtype=torch.complex64, device=dev) \
            if want_E else None
        st = torch.empty((max(n_iter, 1), 4), dtype=torch.float32,
                         device=dev) if want_stats else None
        params = WgsParams(float(power), int(fix_phase_after))
        self._stream()
        check(lib.ash_wgs_iterate(self._h, _ptr(phase), _ptr(weights),
                                  int(n_iter), ctypes.byref(params), _ptr(E),
                                  _ptr(st)), "ash_wgs_iterate", self._h)
        if st is not None:
            st = st[:n_iter]
        return phase, weights, E, st

    def fixed_phases(self, out=None):
        """The stored farfield phases (turns), for checkpoints."""
        if out is None:
            out = torch.empty(self.N, dtype=torch.float32,
                              device="cuda:%d" % self.device)
        _dev(out, torch.float32, (self.N,), "out", self.device)
        self._stream()
        check(lib.ash_get_fixed_phases(self._h, _ptr(out)),
              "ash_get_fixed_phases", self._h)
        return out

    def set_fixed_phases(self, psi):
        """Restore stored farfield phases (turns) from a checkpoint."""
        _dev(psi, torch.float32, (self.N,), "psi", self.device)
        self._stream()
        check(lib.ash_set_fixed_phases(self._h, _ptr(psi)),
              "ash_set_fixed_phases", self._h)

    def wgs_feedback(self, phase, measured, weights=None, power=1.0,
                     fix_phase_after=0, want_E=True, want_stats=True):
        """One weighted-GS iteration whose weights follow the measured spot
        amplitudes; phase and weights are updated in place.

        Returns (phase, weights, E, stats[4]) (E and stats of the model)."""
        _dev(phase, torch.float32, (self.ny, self.nx), "phase", self.device)
        _dev(measured, torch.float32, (self.N,), "measured", self.device)
        dev = "cuda:%d" % self.device
        if weights is None:
            weights = torch.ones(self.N, dtype=torch.float32, device=dev)
        _dev(weights, torch.float32, (self.N,), "weights", self.device)
        E = torch.empty(self.N, dtype=torch.complex64, device=dev) \
            if want_E else None
        st = torch.empty(4, dtype=torch.float32, device=dev) \
            if want_stats else None
        params = WgsParams(float(power), int(fix_phase_after))
        self._stream()
        check(lib.ash_wgs_feedback(self._h, _ptr(phase), _ptr(weights),
                                   _ptr(measured), ctypes.byref(params),
                                   _ptr(E), _ptr(st)),
              "ash_wgs_feedback", self._h)
        return phase, weights, E, st

    # -- differentiable form ----------------------------------------------
    def phase_grad(self, phase, G, out=None):
        """Im(conj(f) sum_n G_n exp(+i theta_n)), f = A exp(i phase): the
        phase gradient of a real loss whose field gradient is G."""
        P = (self.ny, self.nx)
        _dev(phase, torch.float32, P, "phase", self.device)
        _dev(G, torch.complex64, (self.N,), "G", self.device)
        if out is None:
            out = torch.empty(P, dtype=torch.float32,
                              device="cuda:%d" % self.device)
        _dev(out, torch.float32, P, "out", self.device)
        self._stream()
        check(lib.ash_phase_grad(self._h, _ptr(phase), _ptr(G), _ptr(out)),
              "ash_phase_grad", self._h)
        return out

    def forward_moments(self, phase, out=None):
        """M[k, d] = sum_x Z_d(x) f(x) exp(-i theta_k(x)), f = A exp(i phase):
        dE_k/dw[k, d] = -i M[k, d]."""
        _dev(phase, torch.float32, (self.ny, self.nx), "phase", self.device)
        if out is None:
            out = torch.empty((self.N, self.D), dtype=torch.complex64,
                              device="cuda:%d" % self.device)
        _dev(out, torch.complex64, (self.N, self.D), "out", self.device)
        self._stream()
        check(lib.ash_forward_moments(self._h, _ptr(phase), _ptr(out)),
              "ash_forward_moments", self._h)
        return out

    def coef_grad(self, phase, G, out=None):
        """dL/dw[k, d] = Im(conj(G_k) M[k, d]) for the field gradient G."""
        _dev(phase, torch.float32, (self.ny, self.nx), "phase", self.device)
        _dev(G, torch.complex64, (self.N,), "G", self.device)
        if out is None:
            out = torch.empty((self.N, self.D), dtype=torch.float32,
                              device="cuda:%d" % self.device)
        _dev(out, torch.float32, (self.N, self.D), "out", self.device)
        self._stream()
        check(lib.ash_coef_grad(self._h, _ptr(phase), _ptr(G), _ptr(out)),
              "ash_coef_grad", self._h)
        return out

    def window_strehl(self, phase, n_windows, win, out=None):
        """S' = max |E|^2 / sum |E|^2 per window of win*win consecutive
        spots (the spots set by spot_quality / window_coefficients)."""
        _dev(phase, torch.float32, (self.ny, self.nx), "phase", self.device)
        if out is None:
            out = torch.empty(n_windows, dtype=torch.float32,
                              device="cuda:%d" % self.device)
        _dev(out, torch.float32, (n_windows,), "out", self.device)
        self._stream()
        check(lib.ash_window_strehl(self._h, _ptr(phase), int(n_windows),
                                    int(win), _ptr(out)),
              "ash_window_strehl", self._h)
        return out

    def adam(self, phase, n_steps, m=None, v=None, step0=0, lr=0.05,
             betas=(0.9, 0.999), eps=1e-8, tv_weight=1e-3, tv_eps=1e-3,
             want_loss=True, want_E=False):
        """n_steps Adam updates of the spot-amplitude loss with TV; phase,
        m and v are updated in place.  Returns (phase, m, v, losses, E)."""
        P = (self.ny, self.nx)
        dev = "cuda:%d" % self.device
        _dev(phase, torch.float32, P, "phase", self.device)
        if m is None:
            m = torch.zeros(P, dtype=torch.float32, device=dev)
        if v is None:
            v = torch.zeros(P, dtype=torch.float32, device=dev)
        _dev(m, torch.float32, P, "m", self.device)
        _dev(v, torch.float32, P, "v", self.device)
        loss = torch.empty(max(n_steps, 1), dtype=torch.float32,
                           device=dev) if want_loss else None
        E = torch.empty(self.N, dtype=torch.complex64, device=dev) \
            if want_E else None
        prm = AdamParams(lr, betas[0], betas[1], eps, tv_weight, tv_eps)
        self._stream()
        check(lib.ash_adam_iterate(self._h, _ptr(phase), _ptr(m), _ptr(v),
                                   int(step0), int(n_steps),
                                   ctypes.byref(prm), _ptr(loss), _ptr(E)),
              "ash_adam_iterate", self._h)
        if loss is not None:
            loss = loss[:n_steps]
        return phase, m, v, loss, E


class Propagate(torch.autograd.Function):
    """E = forward transform of A exp(i phase), differentiable in phase.

    The backward is the library's adjoint with the phase-gradient epilogue:
    grad_phase = Im(conj(f) sum_n G_n exp(+i theta_n)), where G is torch's
    gradient of the loss with respect to the complex E.  It needs the
    context's basis and spots of the forward: a set_basis or set_spots
    between the two makes the backward raise."""

    @staticmethod
    def forward(ctx, phase, context):
        ctx.context = context
        ctx.generation = context.generation
        ctx.save_for_backward(phase)
        return context.forward(phase=phase.contiguous())

    @staticmethod
    def backward(ctx, grad_E):
        if ctx.context.generation != ctx.generation:
            raise RuntimeError(
                "propagate: the context's basis or spots changed between the "
                "forward and the backward; the gradient would use the new ones")
        (phase,) = ctx.saved_tensors
        G = grad_E.to(torch.complex64).contiguous()
        return ctx.context.phase_grad(phase.contiguous(), G), None


class PropagateSpots(torch.autograd.Function):
    """E = forward transform of A exp(i phase) with kernel coefficients w,
    differentiable in phase and in w.

    The forward sets the context's spots to w (keeping its targets); the
    backward returns the phase gradient of Propagate and
    dL/dw[k, d] = Im(conj(G_k) M[k, d]) from the library's moment
    transform (ash_coef_grad).  If the context's spots changed after the
    forward (another propagate with other w, say), the backward sets them
    back to this forward's w and targets first; a changed basis raises."""

    @staticmethod
    def forward(ctx, phase, w, context):
        context.set_spots(w.detach().to("cpu", torch.float64).numpy(),
                          context.target)
        ctx.context = context
        ctx.generation = context.generation
        ctx.basis_generation = context.basis_generation
        ctx.target = context.target
        ctx.save_for_backward(phase, w)
        return context.forward(phase=phase.contiguous())

    @staticmethod
    def backward(ctx, grad_E):
        phase, w = ctx.saved_tensors
        c = ctx.context
        if c.generation != ctx.generation:
            if c.basis_generation != ctx.basis_generation:
                raise RuntimeError(
                    "propagate: the context's basis changed between the "
                    "forward and the backward")
            c.set_spots(w.detach().to("cpu", torch.float64).numpy(),
                        ctx.target)
            ctx.generation = c.generation
        G = grad_E.to(torch.complex64).contiguous()
        gp = gw = None
        if ctx.needs_input_grad[0]:
            gp = c.phase_grad(phase.contiguous(), G)
        if ctx.needs_input_grad[1]:
            gw = c.coef_grad(phase.contiguous(), G).to(w.device, w.dtype)
        return gp, gw, None


def propagate(phase, context, w=None):
    """Differentiable spot fields of the phase (see Propagate); with w, also
    differentiable in the kernel coefficients (see PropagateSpots)."""
    if w is None:
        return Propagate.apply(phase, context)
    return PropagateSpots.apply(phase, w, context)


def window_coefficients(w, ix, iy, nx, ny, R, step, win):
    """Coefficients of the win x win window points of every spot, `step`
    DFT bins apart on an nx x ny SLM with pupil radius R (see
    ash_window_coefficients): [N * win * win, D] float64."""
    w = np.ascontiguousarray(w, dtype=np.float64)
    N, D = w.shape
    out = np.empty((N * win * win, D), dtype=np.float64)
    check(lib.ash_window_coefficients(N, D, w.ctypes.data, int(ix), int(iy),
                                      int(nx), int(ny), float(R), float(step),
                                      int(win), out.ctypes.data),
          "ash_window_coefficients")
    return out


def spot_quality(camera, phase, w, ix, iy, win=21, step=0.25):
    """S' of win x win farfield windows sampled every `step` DFT bins around
    the spots w, seen through `camera` (a context holding the system's basis
    and amplitude; its spots are replaced by the windows)."""
    ww = window_coefficients(w, ix, iy, camera.nx, camera.ny, camera.R, step,
                             win)
    camera.set_spots(ww)
    return camera.window_strehl(phase, np.asarray(w).shape[0], win)


class Batch:
    """Several holograms (contexts with basis and spots set) whose WGS loops
    run together in persistent launches; see ash_batch_create."""

    def __init__(self, contexts):
        self.members = list(contexts)   # the batch computes in their buffers
        if not self.members:
            raise ValueError("at least one context")
        self.device = self.members[0].device
        H = len(self.members)
        arr = (ctypes.c_void_p * H)(*[c._h.value for c in self.members])
        self._h = ctypes.c_void_p()
        s = torch.cuda.current_stream(self.device).cuda_stream
        rc = lib.ash_batch_create(ctypes.byref(self._h), H, arr,
                                  ctypes.c_void_p(s))
        if rc != 0:
            raise AshError(rc, "ash_batch_create", "")

    def close(self):
        if self._h:
            lib.ash_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc, where):
        if rc != 0:
            raise AshError(rc, where, lib.ash_batch_last_error(self._h).decode())

    def _stream(self):
        s = torch.cuda.current_stream(self.device).cuda_stream
        self._check(lib.ash_batch_set_stream(self._h, ctypes.c_void_p(s)),
                    "ash_batch_set_stream")

    def _ptrs(self, tensors, dtype, shapes, name):
        if len(tensors) != len(self.members):
            raise ValueError("one %s per hologram" % name)
        for t, shp in zip(tensors, shapes):
            _dev(t, dtype, shp, name, self.device)
        return (ctypes.c_void_p * len(tensors))(*[t.data_ptr() for t in tensors])

    def _phases(self, phases):
        return self._ptrs(phases, torch.float32,
                          [(c.ny, c.nx) for c in self.members], "phase")

    def wgs(self, phases, n_iter, weights=None, power=1.0):
        """n_iter WGS iterations of every hologram; phases and weights are
        updated in place.  Returns (phases, weights)."""
        if weights is None:
            weights = [torch.ones(c.N, dtype=torch.float32,
                                  device="cuda:%d" % self.device)
                       for c in self.members]
        ph = self._phases(phases)
        w = self._ptrs(weights, torch.float32, [(c.N,) for c in self.members],
                       "weights")
        params = WgsParams(float(power), 0)
        self._stream()
        self._check(lib.ash_batch_wgs(self._h, ph, w, int(n_iter),
                                      ctypes.byref(params)), "ash_batch_wgs")
        return phases, weights

    def tune(self, phases, table_out=None):
        """Pick the forward range length per record shape by timing."""
        ph = self._phases(phases)
        self._stream()
        self._check(lib.ash_batch_tune(
            self._h, ph, table_out.encode() if table_out else None),
            "ash_batch_tune")
        return self.info()

    def set_form(self, one_launch):
        """One launch per record shape for all iterations (True), or one
        launch per phase of every iteration (False)."""
        self._check(lib.ash_batch_set_form(self._h, int(bool(one_launch))),
                    "ash_batch_set_form")

    def load_tuning(self, table_in):
        self._check(lib.ash_batch_load_tuning(self._h, table_in.encode()),
                    "ash_batch_load_tuning")

    def info(self):
        out = BatchInfo()
        self._check(lib.ash_batch_get_info(self._h, ctypes.byref(out)),
                    "ash_batch_get_info")
        n = out.shapes
        return {"holograms": out.holograms, "shapes": n,
                "groups": list(out.groups)[:min(n, 4)],
                "range_blocks": list(out.range_blocks)[:min(n, 4)],
                "items": out.items,
                "evals_per_transform": out.evals_per_transform,
                "one_launch": bool(out.one_launch),
                "blocks_per_cu": list(out.blocks_per_cu)[:min(n, 4)],
                "grid": list(out.grid)[:min(n, 4)],
                "fused": bool(out.fused)}

    def profile(self, enable=True, categories=None):
        mask = 0
        if enable:
            cats = Context.PROFILE_CATEGORIES if categories is None else categories
            for k in cats:
                mask |= 1 << Context.PROFILE_CATEGORIES.index(k)
        self._check(lib.ash_batch_profile_enable(self._h, mask),
                    "ash_batch_profile_enable")

    def profile_read(self):
        ms = np.zeros(4, dtype=np.float64)
        n = np.zeros(4, dtype=np.int64)
        self._check(lib.ash_batch_profile_read(self._h, ms.ctypes.data,
                                               n.ctypes.data),
                    "ash_batch_profile_read")
        return {k: (float(ms[i]), int(n[i]))
                for i, k in enumerate(Context.PROFILE_CATEGORIES)}
