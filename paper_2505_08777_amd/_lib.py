"""ctypes loader for libash.so (the HIP library built in-tree).

The product path has no CPU fallback: if the library is missing or does not
load, importing this module raises.
"""

import ctypes
import os

# torch brings its own copy of the HIP runtime.  Loading it before libash
# makes libash's libamdhip64 dependency resolve to that same, already loaded
# runtime; two HIP runtimes in one process do not share the device.
import torch  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libash.so")

OK = 0
EINVAL, ESHAPE, ENOTREADY, EUNSUPPORTED, ENOMEM, EHIP = -1, -2, -3, -4, -5, -6

MAX_MODES = 32
MAX_NONLINEAR = 28
MAX_MONOMIALS = 128
MAX_DEGREE = 12
MAX_SIDE = 65536
MAX_SPOTS = 1048576
MAX_PRINCIPAL_MODES = 66


class AshError(RuntimeError):
    def __init__(self, code, where, detail=""):
        self.code = code
        msg = "%s failed: %s (%d)" % (where, strerror(code), code)
        if detail:
            msg += ": " + detail
        super().__init__(msg)


class WgsParams(ctypes.Structure):
    _fields_ = [("power", ctypes.c_float), ("fix_phase_after", ctypes.c_int32)]


class Info(ctypes.Structure):
    _fields_ = [("n_tiles", ctypes.c_int32), ("nonlinear", ctypes.c_int32),
                ("pieces", ctypes.c_int32), ("groups", ctypes.c_int32),
                ("fwd_ranges", ctypes.c_int32), ("rm_bound", ctypes.c_float),
                ("theta_bound", ctypes.c_float),
                ("range_reduce", ctypes.c_int32)]


class AdamParams(ctypes.Structure):
    _fields_ = [("lr", ctypes.c_float), ("beta1", ctypes.c_float),
                ("beta2", ctypes.c_float), ("eps", ctypes.c_float),
                ("tv_weight", ctypes.c_float), ("tv_eps", ctypes.c_float)]


class BatchInfo(ctypes.Structure):
    _fields_ = [("holograms", ctypes.c_int32), ("shapes", ctypes.c_int32),
                ("groups", ctypes.c_int32 * 4),
                ("range_blocks", ctypes.c_int32 * 4),
                ("items", ctypes.c_int64),
                ("evals_per_transform", ctypes.c_double),
                ("one_launch", ctypes.c_int32),
                ("blocks_per_cu", ctypes.c_int32 * 4),
                ("grid", ctypes.c_int32 * 4),
                ("fused", ctypes.c_int32)]


PRECISION_AUTO = 0
PRECISION_FULL = 1


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            "libash.so is not built; run `python -m paper_2505_08777_amd.build` "
            "(hipcc for gfx950) first")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    I = ctypes.c_int
    D = ctypes.c_double
    sig = {
        "ash_version": (I, []),
        "ash_strerror": (ctypes.c_char_p, [I]),
        "ash_last_error": (ctypes.c_char_p, [P]),
        "ash_inject_failure": (I, [I, I]),
        "ash_create": (I, [ctypes.POINTER(P), I, P]),
        "ash_destroy": (I, [P]),
        "ash_set_stream": (I, [P, P]),
        "ash_sync": (I, [P]),
        "ash_zernike_monomials": (I, [I, I, P, P]),
        "ash_principal_modes": (I, [I, I, I, P, P, P, I,
                                    ctypes.POINTER(ctypes.c_int), P, P, P]),
        "ash_set_basis": (I, [P, I, I, D, D, D, I, I, P, P, P]),
        "ash_set_spots": (I, [P, I, P, P]),
        "ash_forward": (I, [P, P, P, P]),
        "ash_forward_noalloc": (I, [P, P, P, P]),
        "ash_adjoint": (I, [P, P, P, P]),
        "ash_wgs_iterate": (I, [P, P, P, I, ctypes.POINTER(WgsParams), P, P]),
        "ash_wgs_feedback": (I, [P, P, P, P, ctypes.POINTER(WgsParams), P, P]),
        "ash_get_fixed_phases": (I, [P, P]),
        "ash_set_fixed_phases": (I, [P, P]),
        "ash_set_precision": (I, [P, I]),
        "ash_get_info": (I, [P, ctypes.POINTER(Info)]),
        "ash_profile_enable": (I, [P, I]),
        "ash_profile_read": (I, [P, P, P]),
        "ash_profile_stride": (I, [P, I]),
        "ash_phase_grad": (I, [P, P, P, P]),
        "ash_forward_moments": (I, [P, P, P]),
        "ash_coef_grad": (I, [P, P, P, P]),
        "ash_window_coefficients": (I, [I, I, P, I, I, I, I, D, D, I, P]),
        "ash_window_strehl": (I, [P, P, I, I, P]),
        "ash_adam_iterate": (I, [P, P, P, P, I, I, ctypes.POINTER(AdamParams),
                                 P, P]),
        "ash_batch_create": (I, [ctypes.POINTER(P), I, P, P]),
        "ash_batch_destroy": (I, [P]),
        "ash_batch_last_error": (ctypes.c_char_p, [P]),
        "ash_batch_set_stream": (I, [P, P]),
        "ash_batch_wgs": (I, [P, P, P, I, ctypes.POINTER(WgsParams)]),
        "ash_batch_tune": (I, [P, P, ctypes.c_char_p]),
        "ash_batch_load_tuning": (I, [P, ctypes.c_char_p]),
        "ash_batch_set_form": (I, [P, I]),
        "ash_batch_get_info": (I, [P, ctypes.POINTER(BatchInfo)]),
        "ash_batch_profile_enable": (I, [P, I]),
        "ash_batch_profile_read": (I, [P, P, P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


lib = _load()


def strerror(code):
    return lib.ash_strerror(code).decode()


INJECT_ALLOC = 1
INJECT_BARRIER = 2


def inject_failure(what, count=1):
    """Arm `count` injected failures of kind `what` (INJECT_ALLOC: device
    allocations fail as out of memory; INJECT_BARRIER: one-launch batch
    calls start with their barrier flag set); count 0 disarms.  For tests
    of the error paths."""
    rc = lib.ash_inject_failure(int(what), int(count))
    if rc != 0:
        raise ValueError("ash_inject_failure: %s" % strerror(rc))


def check(code, where, ctx=None):
    if code != OK:
        detail = lib.ash_last_error(ctx).decode() if ctx else ""
        raise AshError(code, where, detail)
    return code
