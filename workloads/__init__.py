"""Seeded synthetic inputs shaped like the paper's workloads.

This module only draws inputs: spot positions and aberration coefficients,
source amplitudes, target amplitudes and starting phases.  It holds none of
the transform, WGS or gradient arithmetic, and both the oracle tests and the
GPU path consume the arrays it returns.

The paper's calibrations are not published (its data are available on
request), so every workload is a synthetic stand-in with the shapes of the
paper's experiments:

  plain256    256x256 SLM, 25 spots on a 5x5 grid over 80% of the Nyquist
              field, tilt + Noll 4-11 (ANSI 3-9, 12) aberration ~ N(0, 0.5)
  field1024   1024x1024 SLM, 50 isoplanatic patches (10x5) of 8 Zernike
              coefficients ~ N(0, 1), bilinearly interpolated to 400 spots
              on a 20x20 grid over the whole field (stand-in for the 2D
              tweezer array, "A Full-Field 2D Tweezer Array")
  volume1920  1920x1200 SLM, 2000 spots uniform in the Nyquist volume with
              defocus up to +-40 rad at the pupil edge, ANSI 0-14, a smooth
              random aberration field of std 0.8 rad over (x, y, z)
              (stand-in for the volumetric display, "A Corrected Volumetric
              Display")
  grad1024    1024x1024 SLM, 1000 spots in the central 80%, targets
              U[0.5, 1], same basis as field1024, aberration ~ N(0, 0.5)
  batch64     64 holograms, SLM side from {512, 1024, 1536, 2048}, spot
              counts log-uniform in [10, 5000], ANSI tilt + Noll 4-13,
              aberration ~ N(0, 0.7)
  principal1024
              field1024's SLM and 20x20 spot grid with a higher-order
              calibration: 50 patches (10x5) over ANSI 3-27 (radial orders
              2-6) whose coefficients vary smoothly over the field (each a
              random quadratic in the normalised field position, terms of
              std 1.2/(n-1) rad for radial order n), bilinearly interpolated
              to the spots, plus independent calibration noise N(0, 0.05)
              per spot and mode; to be compressed onto K = 8 principal
              isoplanatic modes
              (stand-in for the 44th-order calibration projected onto 8
              principal modes, "A Full-Field 2D Tweezer Array" and Methods,
              "Anisoplanatic Singular Value Decomposition")
  feedback1024
              field1024 as the model, and a simulated optical system for
              the closed loop: the same spots with model errors N(0, 0.1 rad)
              added to each aberration coefficient and per-spot efficiency
              gains U(0.8, 1.2) between the fields and the measured spot
              amplitudes; 30 loop iterations per step, farfield phases fixed
              after 10

Conventions shared with the consumers (and stated on the C ABI):
  pixel (i, j), i the column index (fastest); pupil centre (nx/2, ny/2);
  unit radius R = min(nx, ny)/2; Zernike functions orthonormal on the unit
  disk with ANSI indices, so Z_2 = 2 xh and Z_1 = 2 yh.  A spot at farfield
  position (u, v) in DFT-bin units gets tilt coefficients
  w[ANSI 2] = pi u R / nx and w[ANSI 1] = pi v R / ny (radians), i.e. a
  phase slope of 2 pi u / nx radians per pixel.
  Source amplitude: Gaussian exp(-r^2 / wst^2), r in pixels from the pupil
  centre, wst = 0.4 min(nx, ny).
"""

import math

import numpy as np

BASE_SEED = 2505

NOLL4_11_ANSI = [3, 4, 5, 6, 7, 8, 9, 12]
NOLL4_13_ANSI = [3, 4, 5, 6, 7, 8, 9, 12, 13, 11]

WORKLOADS = ("plain256", "field1024", "volume1920", "grad1024", "batch64",
             "principal1024", "feedback1024")


def geometry(nx, ny):
    return dict(nx=nx, ny=ny, cx=nx / 2.0, cy=ny / 2.0, R=min(nx, ny) / 2.0)


def gaussian_amp(nx, ny):
    g = geometry(nx, ny)
    wst = 0.4 * min(nx, ny)
    i = np.arange(nx) - g["cx"]
    j = np.arange(ny) - g["cy"]
    return np.exp(-(j[:, None] ** 2 + i[None, :] ** 2) / wst ** 2)


def tilt_coefs(u, v, nx, ny):
    """(w[ANSI 1], w[ANSI 2]) in radians for bins (u, v)."""
    R = min(nx, ny) / 2.0
    return np.pi * np.asarray(v) * R / ny, np.pi * np.asarray(u) * R / nx


def random_phase(rng, nx, ny):
    return rng.uniform(-np.pi, np.pi, size=(ny, nx))


def _pack(name, seed, nx, ny, modes, w, t, rng, n_iter, **extra):
    d = dict(name=name, seed=seed, modes=list(modes), w=np.asarray(w, np.float64),
             t=np.asarray(t, np.float64), amp=gaussian_amp(nx, ny),
             phi0=random_phase(rng, nx, ny), n_iter=n_iter)
    d.update(geometry(nx, ny))
    d.update(extra)
    return d


def plain256(seed=None):
    seed = BASE_SEED + 1 if seed is None else seed
    rng = np.random.default_rng(seed)
    n = 256
    g = np.linspace(-0.4 * n, 0.4 * n, 5)
    v, u = np.meshgrid(g, g, indexing="ij")
    u, v = u.ravel(), v.ravel()
    N = u.size
    modes = [1, 2] + NOLL4_11_ANSI
    w = np.zeros((N, len(modes)))
    w[:, 0], w[:, 1] = tilt_coefs(u, v, n, n)
    w[:, 2:] = rng.normal(0.0, 0.5, size=(N, 8))
    return _pack("plain256", seed, n, n, modes, w, np.ones(N), rng, 20,
                 u=u, v=v)


def _bilinear(centres_x, centres_y, vals, qx, qy):
    """vals[iy, ix, :] at centres; clamped bilinear at query points."""
    def locate(c, q):
        q = np.clip(q, c[0], c[-1])
        k = np.clip(np.searchsorted(c, q, side="right") - 1, 0, len(c) - 2)
        fr = (q - c[k]) / (c[k + 1] - c[k])
        return k, fr
    kx, fx = locate(centres_x, qx)
    ky, fy = locate(centres_y, qy)
    v00 = vals[ky, kx]
    v01 = vals[ky, kx + 1]
    v10 = vals[ky + 1, kx]
    v11 = vals[ky + 1, kx + 1]
    fx = fx[:, None]
    fy = fy[:, None]
    return ((1 - fy) * ((1 - fx) * v00 + fx * v01)
            + fy * ((1 - fx) * v10 + fx * v11))


def field1024(seed=None, n=1024):
    seed = BASE_SEED + 2 if seed is None else seed
    rng = np.random.default_rng(seed)
    patches = rng.normal(0.0, 1.0, size=(5, 10, 8))       # [y, x, mode]
    px = -n / 2 + (np.arange(10) + 0.5) * n / 10
    py = -n / 2 + (np.arange(5) + 0.5) * n / 5
    c = -n / 2 + (np.arange(20) + 0.5) * n / 20
    v, u = np.meshgrid(c, c, indexing="ij")
    u, v = u.ravel(), v.ravel()
    N = u.size
    modes = [1, 2] + NOLL4_11_ANSI
    w = np.zeros((N, len(modes)))
    w[:, 0], w[:, 1] = tilt_coefs(u, v, n, n)
    w[:, 2:] = _bilinear(px, py, patches, u, v)
    return _pack("field1024", seed, n, n, modes, w, np.ones(N), rng, 100,
                 u=u, v=v, patches=patches)


def _smooth_field(rng, pts, n_comp=16, std=0.8, corr=0.5):
    """sum of n_comp random Fourier components over pts [M, 3] in [-1, 1]^3."""
    k = rng.normal(0.0, 2 * np.pi / corr, size=(n_comp, 3))
    ph = rng.uniform(0, 2 * np.pi, size=n_comp)
    amp = math.sqrt(2.0 / n_comp) * std
    return amp * np.cos(pts @ k.T + ph).sum(axis=1)


def volume1920(seed=None, nx=1920, ny=1200, N=2000):
    seed = BASE_SEED + 3 if seed is None else seed
    rng = np.random.default_rng(seed)
    u = rng.uniform(-nx / 2, nx / 2, size=N)
    v = rng.uniform(-ny / 2, ny / 2, size=N)
    z = rng.uniform(-1.0, 1.0, size=N)
    modes = list(range(15))
    D = len(modes)
    pts = np.stack([u / (nx / 2), v / (ny / 2), z], axis=1)
    w = np.stack([_smooth_field(rng, pts) for _ in range(D)], axis=1)
    w1, w2 = tilt_coefs(u, v, nx, ny)
    w[:, 1] += w1
    w[:, 2] += w2
    # defocus Z_4 = sqrt(3)(2 rho^2 - 1): edge minus centre = 2 sqrt(3) w_4
    w[:, 4] += 40.0 * z / (2.0 * math.sqrt(3.0))
    return _pack("volume1920", seed, nx, ny, modes, w, np.ones(N), rng, 200,
                 u=u, v=v, z=z)


def grad1024(seed=None, n=1024, N=1000):
    seed = BASE_SEED + 4 if seed is None else seed
    rng = np.random.default_rng(seed)
    u = rng.uniform(-0.4 * n, 0.4 * n, size=N)
    v = rng.uniform(-0.4 * n, 0.4 * n, size=N)
    modes = [1, 2] + NOLL4_11_ANSI
    w = np.zeros((N, len(modes)))
    w[:, 0], w[:, 1] = tilt_coefs(u, v, n, n)
    w[:, 2:] = rng.normal(0.0, 0.5, size=(N, 8))
    t = rng.uniform(0.5, 1.0, size=N)
    d = _pack("grad1024", seed, n, n, modes, w, t, rng, 200, u=u, v=v)
    d["fd_pixels"] = rng.choice(n * n, size=256, replace=False)
    d.update(lr=0.05, betas=(0.9, 0.999), adam_eps=1e-8, lam=1e-3,
             tv_eps=1e-3, fd_h=1e-4)
    return d


def _radial_order(ansi):
    n = 0
    while (n + 1) * (n + 2) // 2 <= ansi:
        n += 1
    return n


def principal1024(seed=None, n=1024, K=8):
    seed = BASE_SEED + 7 if seed is None else seed
    rng = np.random.default_rng(seed)
    aber = list(range(3, 28))
    std = np.array([1.2 / (_radial_order(d) - 1) for d in aber])
    px = -n / 2 + (np.arange(10) + 0.5) * n / 10
    py = -n / 2 + (np.arange(5) + 0.5) * n / 5
    fy, fx = np.meshgrid(py / (n / 2), px / (n / 2), indexing="ij")
    field = np.stack([np.ones_like(fx), fx, fy, fx * fx, fx * fy, fy * fy])
    coef = rng.normal(0.0, 1.0, size=(6, len(aber))) * std
    patches = np.tensordot(field, coef, axes=(0, 0))      # [y, x, mode]
    c = -n / 2 + (np.arange(20) + 0.5) * n / 20
    v, u = np.meshgrid(c, c, indexing="ij")
    u, v = u.ravel(), v.ravel()
    N = u.size
    modes = [1, 2] + aber
    w = np.zeros((N, len(modes)))
    w[:, 0], w[:, 1] = tilt_coefs(u, v, n, n)
    w[:, 2:] = _bilinear(px, py, patches, u, v) \
        + rng.normal(0.0, 0.05, size=(N, len(aber)))
    return _pack("principal1024", seed, n, n, modes, w, np.ones(N), rng, 100,
                 u=u, v=v, K=K)


def feedback1024(seed=None):
    d = field1024()
    d["name"] = "feedback1024"
    rng = np.random.default_rng(BASE_SEED + 8 if seed is None else seed)
    N = d["w"].shape[0]
    w_true = d["w"].copy()
    w_true[:, 2:] += rng.normal(0.0, 0.1, size=(N, w_true.shape[1] - 2))
    d.update(w_true=w_true, gain=rng.uniform(0.8, 1.2, size=N), n_iter=30,
             fix_phase_after=10)
    return d


BATCH_SIDES = (512, 1024, 1536, 2048)


def batch64_specs(seed=None, H=64):
    """Per-hologram (side, N, seed) without the arrays."""
    seed = BASE_SEED + 5 if seed is None else seed
    rng = np.random.default_rng(seed)
    sides = rng.choice(BATCH_SIDES, size=H)
    Ns = np.rint(np.exp(rng.uniform(math.log(10), math.log(5000), size=H)))
    seeds = rng.integers(0, 2 ** 31, size=H)
    return [dict(side=int(s), N=int(n), seed=int(q))
            for s, n, q in zip(sides, Ns.astype(int), seeds)]


def batch64small_specs(seed=None, H=64):
    """64 small holograms (sides 256..512, N log-uniform in [5, 200], 20
    iterations): each one far too small to fill the GPU by itself."""
    seed = BASE_SEED + 11 if seed is None else seed
    rng = np.random.default_rng(seed)
    sides = rng.choice((256, 384, 512), size=H)
    Ns = np.rint(np.exp(rng.uniform(math.log(5), math.log(200), size=H)))
    seeds = rng.integers(0, 2 ** 31, size=H)
    return [dict(side=int(s), N=int(n), seed=int(q), n_iter=20)
            for s, n, q in zip(sides, Ns.astype(int), seeds)]


def batch_hologram(spec):
    n, N, seed = spec["side"], spec["N"], spec["seed"]
    rng = np.random.default_rng(seed)
    u = rng.uniform(-0.45 * n, 0.45 * n, size=N)
    v = rng.uniform(-0.45 * n, 0.45 * n, size=N)
    modes = [1, 2] + NOLL4_13_ANSI
    w = np.zeros((N, len(modes)))
    w[:, 0], w[:, 1] = tilt_coefs(u, v, n, n)
    w[:, 2:] = rng.normal(0.0, 0.7, size=(N, len(modes) - 2))
    return _pack("batch64", seed, n, n, modes, w, np.ones(N), rng,
                 spec.get("n_iter", 50), u=u, v=v)


def make(name, seed=None):
    if name == "batch64":
        return [batch_hologram(s) for s in batch64_specs(seed)]
    if name == "batch64small":
        return [batch_hologram(s) for s in batch64small_specs(seed)]
    return {"plain256": plain256, "field1024": field1024,
            "volume1920": volume1920, "grad1024": grad1024,
            "principal1024": principal1024,
            "feedback1024": feedback1024}[name](seed)
