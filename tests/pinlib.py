"""Independent brute-force helpers that pin the oracle (and, through it, the library).

Nothing here calls the oracle's arithmetic: positions, planes, kernels and
transforms are written out again from their definitions in the plainest form
(explicit exponentials, explicit loops over small inputs).
"""
import math

import numpy as np

TWO_PI = 2.0 * math.pi


def direct_centred_idft(g: np.ndarray) -> np.ndarray:
    """O(N^4) F[q,p] = sum_{j,i} g[j,i] exp(+2 pi i ((i-N/2)(p-N/2) + (j-N/2)(q-N/2))/N)."""
    n = g.shape[-1]
    c = np.arange(n) - n // 2
    # phase[q, p, j, i]
    ph = (c[None, None, None, :] * c[None, :, None, None] +
          c[None, None, :, None] * c[:, None, None, None]) / n
    return np.einsum("qpji,ji->qp", np.exp(1j * TWO_PI * ph), g)


def gauss(d, sigma):
    return np.exp(-(np.asarray(d, dtype=np.float64) ** 2) / (2.0 * sigma * sigma))


def kernel_dft(f, nu, support, sigma):
    """K(f, nu) = sum_a G(a - f) exp(2 pi i (a - f) nu): the transform of one visibility's
    footprint at sub-cell offset f, relative to the exact fringe."""
    h = (support - 1) // 2
    a = np.arange(-h, h + 1, dtype=np.float64)
    f = np.asarray(f, dtype=np.float64)[..., None]
    nu = np.asarray(nu, dtype=np.float64)[..., None]
    return (gauss(a - f, sigma) * np.exp(1j * TWO_PI * (a - f) * nu)).sum(axis=-1)


def c_closed_form(nu, support, sigma):
    """int_{-S/2}^{S/2} exp(-d^2/2s^2) cos(2 pi nu d) dd
    = s sqrt(2 pi) exp(-2 pi^2 s^2 nu^2) Re erf((S/2 - 2 pi i nu s^2)/(s sqrt 2))."""
    from scipy.special import erf
    nu = np.asarray(nu, dtype=np.float64)
    a = support / 2.0
    z = (a - 1j * TWO_PI * nu * sigma * sigma) / (sigma * math.sqrt(2.0))
    return sigma * math.sqrt(TWO_PI) * np.exp(-2 * math.pi ** 2 * sigma ** 2 * nu ** 2) * erf(z).real


def kernel_eps(support, sigma, nu_max, n_f=1201, n_nu=257):
    """sup over offsets f in [-1/2, 1/2] and |nu| <= nu_max of |K(f,nu)/C(nu) - 1|."""
    f = np.linspace(-0.5, 0.5, n_f)
    nu = np.linspace(-nu_max, nu_max, n_nu)
    k = kernel_dft(f[:, None], nu[None, :], support, sigma)
    c = c_closed_form(nu, support, sigma)
    return float(np.abs(k / c[None, :] - 1.0).max())


def positions(uvw_lambda, n, cell):
    """x = u * (N dl) + N/2 (two roundings, as the method states)."""
    scale = n * cell
    x = uvw_lambda[:, 0] * scale + n / 2
    y = uvw_lambda[:, 1] * scale + n / 2
    return x, y


def planes(w, w_min, w_max, n_w):
    dw = (w_max - w_min) / n_w
    if dw == 0.0:
        return np.zeros(len(w), dtype=np.int64), np.full(len(w), w_min)
    k = np.minimum(n_w - 1, np.floor((w - w_min) / dw)).astype(np.int64)
    return k, w_min + (k + 0.5) * dw


def n_minus_1_ld(eta):
    """sqrt(1 - eta) - 1 evaluated with 50-digit arithmetic (mpmath)."""
    import mpmath
    mpmath.mp.dps = 50
    return np.array([float(mpmath.sqrt(1 - mpmath.mpf(float(e))) - 1) for e in eta])


def quantised_dft(uvw_lambda, vis, wts, w_min, w_max, n_w, n, cell, pix_q, pix_p):
    """D_q(q,p) = sum W Re(V exp(2 pi i (u l + v m + w_k (n-1)))) / sum W: the direct
    transform with each w replaced by its plane's w_k (no gridding kernel)."""
    k, wk = planes(uvw_lambda[:, 2], w_min, w_max, n_w)
    l = (np.asarray(pix_p) - n / 2) * cell
    m = (np.asarray(pix_q) - n / 2) * cell
    nm1 = np.sqrt(1.0 - l * l - m * m) - 1.0
    out = np.empty(len(l))
    for t in range(len(l)):
        ph = TWO_PI * (uvw_lambda[:, 0] * l[t] + uvw_lambda[:, 1] * m[t] + wk * nm1[t])
        out[t] = (wts * (vis * np.exp(1j * ph)).real).sum() / wts.sum()
    return out


def exact_dft(uvw_lambda, vis, wts, n, cell, pix_q, pix_p):
    """Eq. 1 inverted directly: D(q,p) = sum W Re(V exp(2 pi i (u l + v m + w (n-1)))) / sum W."""
    l = (np.asarray(pix_p) - n / 2) * cell
    m = (np.asarray(pix_q) - n / 2) * cell
    nm1 = np.sqrt(1.0 - l * l - m * m) - 1.0
    out = np.empty(len(l))
    for t in range(len(l)):
        ph = TWO_PI * (uvw_lambda[:, 0] * l[t] + uvw_lambda[:, 1] * m[t] + uvw_lambda[:, 2] * nm1[t])
        out[t] = (wts * (vis * np.exp(1j * ph)).real).sum() / wts.sum()
    return out
