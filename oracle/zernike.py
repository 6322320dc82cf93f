"""Zernike polynomials by the radial formula, in float64 (test infrastructure).

The paper indexes each polynomial Z_d = Z_n^l by a single ANSI index d and
notes x ~ Z_2 = Z_1^1, y ~ Z_1 = Z_1^{-1}, defocus ~ Z_4 = Z_2^0 and
spherical Z_12 = Z_4^0 ("Aberration-Space Holography", modal-expansion
paragraph).  The paper does not fix a normalisation; the reading taken here
is the orthonormal one on the unit disk (mean of Z_i Z_j over the disk is
delta_ij), which makes Z_1^1 = 2x exactly as in the paper's tilt statement.

Evaluation is in polar coordinates, rho = hypot(x, y) and angle
atan2(y, x), with the textbook radial sum; it is applied at every point,
including rho > 1 (the pupil support comes from the source amplitude).
"""

from math import factorial, sqrt

import numpy as np


def ansi_to_nm(d):
    """ANSI single index d -> (radial order n, azimuthal order m)."""
    if d < 0:
        raise ValueError("ANSI index must be >= 0")
    n = 0
    while (n + 1) * (n + 2) // 2 <= d:
        n += 1
    m = 2 * d - n * (n + 2)
    return n, m


def nm_to_ansi(n, m):
    if abs(m) > n or (n - m) % 2:
        raise ValueError("invalid (n, m)")
    return (n * (n + 2) + m) // 2


def noll_to_nm(j):
    """Noll index j (1-based) -> (n, m).

    Noll's ordering: increasing n, then increasing |m|; for m != 0 the pair
    of indices is split so that the even index carries the cosine term
    (m > 0) and the odd index the sine term (m < 0).
    """
    if j < 1:
        raise ValueError("Noll index must be >= 1")
    k = 1
    n = 0
    while True:
        for am in range(n % 2, n + 1, 2):
            if am == 0:
                if k == j:
                    return n, 0
                k += 1
            else:
                for idx in (k, k + 1):
                    if idx == j:
                        return n, (am if idx % 2 == 0 else -am)
                k += 2
        n += 1


def noll_to_ansi(j):
    return nm_to_ansi(*noll_to_nm(j))


def radial(n, am, rho):
    """R_n^{|m|}(rho) by the finite sum over s (textbook radial formula)."""
    out = np.zeros_like(rho, dtype=np.float64)
    for s in range((n - am) // 2 + 1):
        c = ((-1) ** s * factorial(n - s)
             / (factorial(s) * factorial((n + am) // 2 - s)
                * factorial((n - am) // 2 - s)))
        out = out + c * rho ** (n - 2 * s)
    return out


def zernike_nm(n, m, x, y):
    """Orthonormal Zernike Z_n^m at Cartesian points (x, y) (float64)."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    rho = np.hypot(x, y)
    ang = np.arctan2(y, x)
    norm = sqrt(2.0 * (n + 1) / (2.0 if m == 0 else 1.0))
    r = radial(n, abs(m), rho)
    if m > 0:
        return norm * r * np.cos(m * ang)
    if m < 0:
        return norm * r * np.sin(-m * ang)
    return norm * r


class ZernikeBasis:
    """Basis {Z_d} for a list of ANSI indices, evaluated by the radial formula."""

    def __init__(self, ansi):
        self.ansi = [int(d) for d in ansi]
        self.nm = [ansi_to_nm(d) for d in self.ansi]

    @property
    def D(self):
        return len(self.ansi)

    def evaluate(self, x, y):
        """Return Z with shape (D,) + x.shape."""
        return np.stack([zernike_nm(n, m, x, y) for n, m in self.nm])


class MonomialBasis:
    """A basis given directly as Z_d(x, y) = sum_k a[d, k] x^p_k y^q_k.

    This is the form in which the paper's GPU implementation receives the
    basis (Methods, "Computational Scaling": the monomial expansion of each
    basis function).  The oracle evaluates it term by term in float64; it is
    used for non-Zernike test bases such as {x^2, y^2}.
    """

    def __init__(self, powers, coefs):
        self.powers = [(int(p), int(q)) for p, q in powers]
        self.coefs = np.asarray(coefs, dtype=np.float64)
        if self.coefs.ndim != 2 or self.coefs.shape[1] != len(self.powers):
            raise ValueError("coefs must be [D, n_mono]")

    @property
    def D(self):
        return self.coefs.shape[0]

    def evaluate(self, x, y):
        x = np.asarray(x, dtype=np.float64)
        y = np.asarray(y, dtype=np.float64)
        out = np.zeros((self.D,) + x.shape)
        for k, (p, q) in enumerate(self.powers):
            mono = x ** p * y ** q
            for d in range(self.D):
                if self.coefs[d, k] != 0.0:
                    out[d] += self.coefs[d, k] * mono
        return out
