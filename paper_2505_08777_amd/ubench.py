"""ctypes binding of libash_ubench.so: the measured issue costs behind the
transforms' issue ceiling (see include/ash_ubench.h)."""

import ctypes
import os

import torch  # noqa: F401  (the HIP runtime the library resolves to)

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libash_ubench.so")


class IssueRates(ctypes.Structure):
    _fields_ = [("simds", ctypes.c_int), ("nominal_clock_hz", ctypes.c_double),
                ("fma_cycles", ctypes.c_double),
                ("trans_cycles", ctypes.c_double),
                ("mfma_cycles", ctypes.c_double), ("ms", ctypes.c_float * 3)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError("libash_ubench.so is not built; run "
                          "`python paper_2505_08777_amd/build.py` first")
    lib = ctypes.CDLL(LIB_PATH)
    lib.ash_ubench_issue.restype = ctypes.c_int
    lib.ash_ubench_issue.argtypes = [ctypes.c_int, ctypes.c_int,
                                     ctypes.POINTER(IssueRates)]
    lib.ash_ubench_mix.restype = ctypes.c_int
    lib.ash_ubench_mix.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                   ctypes.c_int, ctypes.c_int,
                                   ctypes.POINTER(ctypes.c_double)]
    return lib


def issue_rates(device=0, waves_per_simd=4):
    """{'fma', 'trans', 'mfma'} cycles per wave64 instruction per SIMD at the
    nominal clock, with the SIMD count and the clock."""
    out = IssueRates()
    rc = _load().ash_ubench_issue(int(device), int(waves_per_simd),
                                  ctypes.byref(out))
    if rc != 0:
        raise RuntimeError("ash_ubench_issue failed (%d)" % rc)
    return {"fma": out.fma_cycles, "trans": out.trans_cycles,
            "mfma": out.mfma_cycles, "simds": out.simds,
            "nominal_clock_hz": out.nominal_clock_hz,
            "waves_per_simd": int(waves_per_simd),
            "launch_ms": [float(x) for x in out.ms]}


def mix_ceiling(groups, reduce=False, moments=False, device=0,
                occupancies=(4, 5, 6, 8)):
    """Evaluations/s of the transforms' irreducible instruction mix (see
    ash_ubench_mix), the best over the given waves per SIMD, and that
    occupancy."""
    lib = _load()
    best, best_w = 0.0, None
    for w in occupancies:
        v = ctypes.c_double()
        rc = lib.ash_ubench_mix(int(device), int(groups), int(bool(reduce)),
                                int(bool(moments)), int(w), ctypes.byref(v))
        if rc != 0:
            raise RuntimeError("ash_ubench_mix failed (%d)" % rc)
        if v.value > best:
            best, best_w = v.value, w
    return best, best_w
