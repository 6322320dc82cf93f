"""Spot-amplitude loss, its analytic phase gradient and central differences.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper optimises the complex Fourier weights by gradient descent through
its cached transforms for precision targets (Methods, "Computational
Scaling", last paragraph) but gives no loss.  The reading used here:

  normalised fields  Eh_k = E_k / s,  s = sqrt(P * sum_x A^2 / N)
                     (a lossless, uniform split gives |Eh_k|^2 = 1)
  spot term          L_spot = sum_k (|Eh_k|^2 - t_k)^2
  TV term            TV = (1/P) sum_x sqrt(dx^2 + dy^2 + eps^2),
                     dx = wrap(phi[j, i+1] - phi[j, i]) (0 on the last
                     column), dy likewise along j, wrap into (-pi, pi]
  total              L = L_spot + lam * TV

Derivatives, with f = A exp(i phi), theta_k the kernel phase:

  dE_k/dphi(x) = i f(x) exp(-i theta_k(x))
  dL_spot/dphi(x) = Im( conj(f(x)) * sum_k G_k exp(+i theta_k(x)) ),
                    G_k = 4 (|Eh_k|^2 - t_k) Eh_k / s
  dTV/dphi        differentiates each square root through the two forward
                  differences it contains (wrap has unit slope).

Central differences at selected pixels use the exact field update
E_k(phi + h e_x) = E_k + A(x) exp(-i theta_k(x)) (exp(i(phi_x + h)) -
exp(i phi_x)), which costs O(N D) per pixel, plus the change of the few TV
terms that contain phi_x.
"""

import numpy as np

from .transform import forward, adjoint, kernel_phase


def spot_norm(amp, N):
    amp = np.asarray(amp, dtype=np.float64)
    return np.sqrt(amp.size * np.sum(amp ** 2) / N)


def spot_loss(E, t, s):
    Eh = np.asarray(E) / s
    return float(np.sum((np.abs(Eh) ** 2 - np.asarray(t)) ** 2))


def _wrap(d):
    # into (-pi, pi]
    return np.pi - np.mod(np.pi - d, 2 * np.pi)


def _diffs(phi):
    dx = np.zeros_like(phi)
    dy = np.zeros_like(phi)
    dx[:, :-1] = _wrap(phi[:, 1:] - phi[:, :-1])
    dy[:-1, :] = _wrap(phi[1:, :] - phi[:-1, :])
    return dx, dy


def tv_loss(phi, eps=1e-3):
    phi = np.asarray(phi, dtype=np.float64)
    dx, dy = _diffs(phi)
    return float(np.sum(np.sqrt(dx ** 2 + dy ** 2 + eps ** 2)) / phi.size)


def tv_grad(phi, eps=1e-3):
    phi = np.asarray(phi, dtype=np.float64)
    dx, dy = _diffs(phi)
    q = np.sqrt(dx ** 2 + dy ** 2 + eps ** 2)
    gx = dx / q
    gy = dy / q
    g = -gx - gy
    g[:, 1:] += gx[:, :-1]
    g[1:, :] += gy[:-1, :]
    return g / phi.size


def total_loss(phi, amp, t, w, basis, geom, lam=1e-3, eps=1e-3, workers=None):
    """Returns (L, E)."""
    phi = np.asarray(phi, dtype=np.float64)
    f = np.asarray(amp, dtype=np.float64) * np.exp(1j * phi)
    E = forward(f, w, basis, geom, workers=workers)
    s = spot_norm(amp, len(t))
    return spot_loss(E, t, s) + lam * tv_loss(phi, eps), E


def loss_grad(phi, amp, t, w, basis, geom, lam=1e-3, eps=1e-3, workers=None,
              E=None):
    """Analytic dL/dphi (shape of phi). Returns (grad, L, E)."""
    phi = np.asarray(phi, dtype=np.float64)
    amp = np.asarray(amp, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    f = amp * np.exp(1j * phi)
    if E is None:
        E = forward(f, w, basis, geom, workers=workers)
    s = spot_norm(amp, len(t))
    Eh = E / s
    G = 4.0 * (np.abs(Eh) ** 2 - t) * Eh / s
    h = adjoint(G, w, basis, geom, workers=workers)
    grad = np.imag(np.conj(f) * h) + lam * tv_grad(phi, eps)
    L = spot_loss(E, t, s) + lam * tv_loss(phi, eps)
    return grad, L, E


def _tv_terms_at(phi, j, i, eps):
    """Sum of the TV square roots that contain phi[j, i] (unscaled)."""
    ny, nx = phi.shape
    tot = 0.0
    for (jj, ii) in ((j, i), (j, i - 1), (j - 1, i)):
        if jj < 0 or ii < 0:
            continue
        dx = _wrap(phi[jj, ii + 1] - phi[jj, ii]) if ii + 1 < nx else 0.0
        dy = _wrap(phi[jj + 1, ii] - phi[jj, ii]) if jj + 1 < ny else 0.0
        tot += np.sqrt(dx * dx + dy * dy + eps * eps)
    return tot


def fd_grad(phi, pixels, amp, t, w, basis, geom, h=1e-4, lam=1e-3,
            eps=1e-3, E=None, workers=None):
    """Central differences (L(phi + h e_x) - L(phi - h e_x)) / 2h at pixels.

    ``pixels`` are flat indices.  Uses the O(N) exact field update.
    """
    phi = np.array(phi, dtype=np.float64)   # private copy: perturbed below
    amp = np.asarray(amp, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    if E is None:
        E = forward(amp * np.exp(1j * phi), w, basis, geom, workers=workers)
    s = spot_norm(amp, len(t))
    P = phi.size
    out = np.zeros(len(pixels))
    for q, p in enumerate(pixels):
        j, i = divmod(int(p), geom.nx)
        th = kernel_phase(w, basis, geom, np.array([p]))[:, 0]
        Kc = np.exp(-1j * th)
        a = amp[j, i]
        base = np.exp(1j * phi[j, i])
        vals = []
        for sgn in (+1.0, -1.0):
            Ep = E + a * Kc * (np.exp(1j * (phi[j, i] + sgn * h)) - base)
            ls = spot_loss(Ep, t, s)
            old = phi[j, i]
            tv_old = _tv_terms_at(phi, j, i, eps)
            phi[j, i] = old + sgn * h
            tv_new = _tv_terms_at(phi, j, i, eps)
            phi[j, i] = old
            vals.append((ls, tv_new - tv_old))
        (lp, dtp), (lm, dtm) = vals
        out[q] = ((lp - lm) + lam * (dtp - dtm) / P) / (2 * h)
    return out


def adam_step(phi, grad, m, v, step, lr=0.05, beta1=0.9, beta2=0.999,
              eps=1e-8):
    """One Adam update (Kingma and Ba, 2015) of the phase.

    ``step`` is the 1-based index of this update.  The moment estimates are
    exponential averages of the gradient and of its square; each is divided
    by one minus its decay rate to the power ``step`` to remove the bias of
    the zero start, and the phase moves by lr * m_hat / (sqrt(v_hat) + eps).
    Returns (phi, m, v), new arrays.
    """
    g = np.asarray(grad, dtype=np.float64)
    m = beta1 * np.asarray(m, dtype=np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, dtype=np.float64) + (1.0 - beta2) * g * g
    m_hat = m / (1.0 - beta1 ** step)
    v_hat = v / (1.0 - beta2 ** step)
    phi = np.asarray(phi, dtype=np.float64) - lr * m_hat / (np.sqrt(v_hat) + eps)
    return phi, m, v


def adam_run(phi, amp, t, w, basis, geom, n_steps, lr=0.05, betas=(0.9, 0.999),
             eps=1e-8, lam=1e-3, tv_eps=1e-3, workers=None):
    """n_steps Adam updates of L from phi with zero moments.

    Returns (phi, m, v, losses) with losses[s] = L at the phase before
    update s + 1."""
    phi = np.asarray(phi, dtype=np.float64)
    m = np.zeros_like(phi)
    v = np.zeros_like(phi)
    losses = []
    for s in range(1, n_steps + 1):
        g, L, _ = loss_grad(phi, amp, t, w, basis, geom, lam=lam, eps=tv_eps,
                            workers=workers)
        losses.append(L)
        phi, m, v = adam_step(phi, g, m, v, s, lr, betas[0], betas[1], eps)
    return phi, m, v, np.array(losses)


# ---------------------------------------------------------------------------
# Gradients with respect to the kernel coefficients w[k, d]
# ---------------------------------------------------------------------------
# The paper moves spots in aberration space by changing w (Methods,
# "Computational Scaling": agile updates of the N x D matrix) and fits
# aberrations in situ; differentiating the spot fields by w gives
#
#   dE_k/dw[k, d] = -i M[k, d],   M[k, d] = sum_x Z_d(x) f(x) exp(-i theta_k(x))
#
# (each E_k depends on its own row w[k] only), so for a real loss with
# G_k = dL/dRe E_k + i dL/dIm E_k
#
#   dL/dw[k, d] = Re(conj(G_k) dE_k/dw[k, d]) = Im(conj(G_k) M[k, d]).

def forward_moments(f, w, basis, geom, spots=None, workers=None):
    """M[k, d] = sum_x Z_d(x) f(x) exp(-i theta_k(x)), complex128 [N, D]
    (rows of the `spots` subset only, if given)."""
    f = np.asarray(f, dtype=np.complex128).reshape(-1)
    w = np.asarray(w, dtype=np.float64)
    xh, yh = geom.coords(np.arange(geom.P))
    Z = basis.evaluate(xh, yh)                             # [D, P]
    cols = [forward(Z[d] * f, w, basis, geom, spots=spots, workers=workers)
            for d in range(Z.shape[0])]
    return np.stack(cols, axis=1)


def coef_grad(f, w, basis, geom, G, spots=None, workers=None):
    """dL/dw[k, d] = Im(conj(G_k) M[k, d]) for the field gradient G
    (G indexed like the rows returned)."""
    M = forward_moments(f, w, basis, geom, spots, workers)
    G = np.asarray(G, dtype=np.complex128).reshape(-1)
    return np.imag(np.conj(G)[:, None] * M)
