"""Principal isoplanatic modes: the SVD rotation of the aberration basis.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Methods, "Anisoplanatic Singular Value Decomposition": the N x D matrix W of
spot coefficients is factored W = U S V^T.  The columns of V rotate the
Zernike basis into principal isoplanatic modes, ordered by singular value;
zeroing all but the K largest singular values gives the truncated correction
(the paper keeps K = 8 of a 44th-order calibration).  The modal-expansion
paragraph of "Computational Scaling" notes that such a basis lowers D, the
per-evaluation cost.

Reading taken here: the decomposition acts on the coefficients of the
non-linear modes only.  Piston and the tilts carry each spot's constant and
its position in the farfield, which are not a low-rank correction; they are
kept exactly.  With R the non-linear modes and V_K the first K columns of V
for W_R = W[:, R]:

    basis_K = [Z_d for linear d] + [B_j = sum_{d in R} V[d, j] Z_d, j < K]
    w_K     = [W[:, linear], W_R V_K]

so the kernel phase becomes sum_d W_d Z_d with W_R replaced by its best
rank-K approximation W_R V_K V_K^T (Eckart-Young).  The product W_R V_K V_K^T
does not depend on the signs of the singular vectors; V_K itself does.
"""

import numpy as np

from .zernike import ZernikeBasis, MonomialBasis


def linear_modes(basis):
    """Boolean mask of the modes that are affine in (x, y)."""
    if isinstance(basis, ZernikeBasis):
        return np.array([n <= 1 for n, _ in basis.nm])
    if isinstance(basis, MonomialBasis):
        deg = np.array([p + q for p, q in basis.powers])
        return np.array([bool(np.all(deg[basis.coefs[d] != 0.0] <= 1))
                         for d in range(basis.D)])
    if isinstance(basis, RotatedBasis):
        return np.array([True] * len(basis.keep) + [False] * basis.V.shape[1])
    raise TypeError("unknown basis type")


class RotatedBasis:
    """[base modes `keep`] followed by the rotated modes Z[rot]^T V."""

    def __init__(self, base, keep, rot, V):
        self.base = base
        self.keep = np.asarray(keep, dtype=np.int64)
        self.rot = np.asarray(rot, dtype=np.int64)
        self.V = np.asarray(V, dtype=np.float64)      # [len(rot), K]

    @property
    def D(self):
        return len(self.keep) + self.V.shape[1]

    def evaluate(self, x, y):
        Z = self.base.evaluate(x, y)
        B = np.tensordot(self.V.T, Z[self.rot], axes=1)
        return np.concatenate([Z[self.keep], B], axis=0)


def principal_modes(w, basis, K):
    """Rotate the non-linear modes of `basis` onto the K leading principal
    modes of the coefficient matrix w [N, D].

    Returns (w_K [N, n_lin + K], basis_K, sigma [n_rot]) with the singular
    values of W_R in descending order (zeros where N < n_rot).
    """
    w = np.asarray(w, dtype=np.float64)
    lin = linear_modes(basis)
    keep = np.flatnonzero(lin)
    rot = np.flatnonzero(~lin)
    n_rot = rot.size
    if not 0 <= K <= n_rot:
        raise ValueError("K must be in [0, %d]" % n_rot)
    WR = w[:, rot]
    _, s, Vt = np.linalg.svd(WR, full_matrices=True)
    sigma = np.zeros(n_rot)
    sigma[:s.size] = s
    VK = Vt[:K].T                                     # [n_rot, K]
    wK = np.concatenate([w[:, keep], WR @ VK], axis=1)
    return wK, RotatedBasis(basis, keep, rot, VK), sigma
