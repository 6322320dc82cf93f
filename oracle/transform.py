"""Compressed forward / adjoint transforms with per-spot kernels (float64).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Definitions ("Aberration-Space Holography", the compressed-sum equations and
the modal-expansion paragraph):

    kernel phase   theta_n(x) = sum_d w[n, d] * Z_d(xh, yh)          (radians)
    kernel         K_n(x)     = exp(-i theta_n(x))
    forward        F_n        = sum_x K_n(x) f(x)
    adjoint        g(x)       = sum_n conj(K_n(x)) y_n

The paper writes both with "proportional to"; the reading taken here is the
unnormalised sums above (the forward matches numpy's ``fft2`` sign and scale
for integer-bin tilts) and the exact conjugate transpose for the adjoint.

Pixel x = (i, j), i the fastest (column) index, flat index p = j*nx + i.
Normalised pupil coordinates: xh = (i - cx)/R, yh = (j - cy)/R, with the
default reading cx = nx/2, cy = ny/2, R = min(nx, ny)/2 (the paper only says
"circular pupil").

The pixel sum is taken over consecutive pixel ranges whose partial sums are
added in order; each range is one numpy matrix product.  Ranges run on a
thread pool, BLAS pinned to one thread per worker.
"""

import os
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass

import numpy as np

try:
    from threadpoolctl import threadpool_limits
except ImportError:  # pragma: no cover
    threadpool_limits = None


@dataclass(frozen=True)
class Geometry:
    nx: int
    ny: int
    cx: float = None
    cy: float = None
    R: float = None

    def __post_init__(self):
        if self.cx is None:
            object.__setattr__(self, "cx", self.nx / 2.0)
        if self.cy is None:
            object.__setattr__(self, "cy", self.ny / 2.0)
        if self.R is None:
            object.__setattr__(self, "R", min(self.nx, self.ny) / 2.0)

    @property
    def P(self):
        return self.nx * self.ny

    def coords(self, flat_idx):
        flat_idx = np.asarray(flat_idx, dtype=np.int64)
        i = flat_idx % self.nx
        j = flat_idx // self.nx
        return (i - self.cx) / self.R, (j - self.cy) / self.R


def _workers(workers):
    if workers is not None:
        return max(1, int(workers))
    try:
        return max(1, len(os.sched_getaffinity(0)))
    except AttributeError:  # pragma: no cover
        return os.cpu_count() or 1


def kernel_phase(w, basis, geom, flat_idx):
    """theta[n, k] = sum_d w[n, d] Z_d(x_k) for the pixels flat_idx."""
    xh, yh = geom.coords(flat_idx)
    Z = basis.evaluate(xh, yh)                     # [D, npix]
    return np.asarray(w, dtype=np.float64) @ Z     # [N, npix]


def _chunks(total, size):
    return [(a, min(a + size, total)) for a in range(0, total, size)]


def _run(tasks, fn, workers):
    nw = _workers(workers)
    if nw == 1 or len(tasks) == 1:
        return [fn(t) for t in tasks]
    if threadpool_limits is not None:
        with threadpool_limits(limits=1):
            with ThreadPoolExecutor(nw) as ex:
                return list(ex.map(fn, tasks))
    with ThreadPoolExecutor(nw) as ex:  # pragma: no cover
        return list(ex.map(fn, tasks))


def forward(f, w, basis, geom, spots=None, pixels=None, workers=None,
            chunk=None):
    """F_n = sum_x exp(-i theta_n(x)) f(x), float64/complex128.

    f       complex nearfield, shape (ny, nx) or (P,)
    w       [N, D] kernel coefficients (radians)
    spots   optional index subset of the N spots to evaluate (outputs are
            independent per spot)
    pixels  optional subset of flat pixel indices to sum over (default: all)
    """
    f = np.asarray(f, dtype=np.complex128).reshape(-1)
    w = np.asarray(w, dtype=np.float64)
    if spots is not None:
        w = w[np.asarray(spots)]
    pix = np.arange(geom.P) if pixels is None else np.asarray(pixels)
    if f.shape[0] != geom.P:
        raise ValueError("f has the wrong size")
    N = w.shape[0]
    if chunk is None:
        chunk = max(256, min(16384, (1 << 24) // max(N, 1)))

    def part(rng):
        a, b = rng
        idx = pix[a:b]
        th = kernel_phase(w, basis, geom, idx)
        return np.exp(-1j * th) @ f[idx]

    parts = _run(_chunks(pix.shape[0], chunk), part, workers)
    out = np.zeros(N, dtype=np.complex128)
    for p in parts:
        out += p
    return out


def adjoint(y, w, basis, geom, pixels=None, workers=None, chunk=None):
    """g(x) = sum_n exp(+i theta_n(x)) y_n, float64/complex128.

    Returns shape (ny, nx) for all pixels, or (len(pixels),) for a subset
    (outputs are independent per pixel).
    """
    y = np.asarray(y, dtype=np.complex128).reshape(-1)
    w = np.asarray(w, dtype=np.float64)
    if y.shape[0] != w.shape[0]:
        raise ValueError("y and w disagree on N")
    pix = np.arange(geom.P) if pixels is None else np.asarray(pixels)
    N = w.shape[0]
    if chunk is None:
        chunk = max(256, min(16384, (1 << 24) // max(N, 1)))

    def part(rng):
        a, b = rng
        th = kernel_phase(w, basis, geom, pix[a:b])
        return y @ np.exp(1j * th)

    parts = _run(_chunks(pix.shape[0], chunk), part, workers)
    g = np.concatenate(parts) if parts else np.zeros(0, np.complex128)
    if pixels is None:
        return g.reshape(geom.ny, geom.nx)
    return g
