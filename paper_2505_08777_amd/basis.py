"""Basis tables for ash_set_basis: Zernike polynomials as monomial sums.

The expansion itself is done by the library (ash_zernike_monomials); this
module only gathers the terms of several modes into one table.
"""

import ctypes

import numpy as np

from ._lib import lib, AshError, MAX_MONOMIALS


def zernike_monomials(ansi):
    """Return (powers [n, 2] int32, coefs [n] float64) for ANSI index."""
    cap = MAX_MONOMIALS
    pw = np.zeros((cap, 2), dtype=np.int32)
    cf = np.zeros(cap, dtype=np.float64)
    n = lib.ash_zernike_monomials(int(ansi), cap, pw.ctypes.data, cf.ctypes.data)
    if n < 0:
        raise AshError(n, "ash_zernike_monomials")
    return pw[:n].copy(), cf[:n].copy()


def zernike_table(modes):
    """Monomial table for the ANSI modes: (mono_pow [M, 2], mono_coef [D, M])."""
    terms = [zernike_monomials(d) for d in modes]
    keys = sorted({(int(p), int(q)) for pw, _ in terms for p, q in pw},
                  key=lambda t: (t[0] + t[1], -t[0]))
    index = {k: i for i, k in enumerate(keys)}
    coef = np.zeros((len(modes), len(keys)), dtype=np.float64)
    for d, (pw, cf) in enumerate(terms):
        for (p, q), c in zip(pw, cf):
            coef[d, index[(int(p), int(q))]] += c
    return np.asarray(keys, dtype=np.int32).reshape(-1, 2), coef


def principal_modes(mono_pow, mono_coef, w, K):
    """Rotate the non-linear modes onto the K leading principal modes of w.

    mono_pow [M, 2], mono_coef [D, M]: the basis; w [N, D]: spot
    coefficients.  Returns (mono_coef_K [D_K, M], w_K [N, D_K],
    sigma [n_rot]) with D_K = (modes kept unchanged) + K; pass them to
    Context.set_basis(mono_pow=mono_pow, mono_coef=mono_coef_K) and
    Context.set_spots(w_K).  See ash_principal_modes in include/ash.h.
    """
    mono_pow = np.ascontiguousarray(mono_pow, dtype=np.int32)
    mono_coef = np.ascontiguousarray(mono_coef, dtype=np.float64)
    w = np.ascontiguousarray(w, dtype=np.float64)
    D, M = mono_coef.shape
    N = w.shape[0]
    if w.ndim != 2 or w.shape[1] != D or mono_pow.shape != (M, 2):
        raise ValueError("w must be [N, D] and mono_pow [M, 2]")
    d_out = ctypes.c_int(0)
    sigma = np.zeros(D, dtype=np.float64)
    mono_out = np.zeros((D, M), dtype=np.float64)
    w_out = np.zeros(N * D, dtype=np.float64)
    rc = lib.ash_principal_modes(N, D, M, mono_pow.ctypes.data,
                                 mono_coef.ctypes.data, w.ctypes.data, int(K),
                                 ctypes.byref(d_out), sigma.ctypes.data,
                                 mono_out.ctypes.data, w_out.ctypes.data)
    if rc != 0:
        raise AshError(rc, "ash_principal_modes")
    Dk = d_out.value
    n_rot = D - (Dk - int(K))
    return (mono_out[:Dk].copy(), w_out[:N * Dk].reshape(N, Dk).copy(),
            sigma[:n_rot].copy())
