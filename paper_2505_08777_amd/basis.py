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
