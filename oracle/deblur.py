"""EPLL with a general degradation operator A: periodic deblurring -- the
reference definition.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
benchmark's CPU-baseline leg may import this module; the restoration library
never does, and this module imports nothing from it.

Alg. 1's image estimation solves (A^t A + beta sigma^2 I) x = A^t y +
beta sigma^2 x~; for a periodic convolution A is diagonal in the Fourier
basis, so the solve is a pointwise division between two 2-D FFTs (Sec. 2.1,
the complexity discussion of the image-estimation step).  Sec. 5
("Parameter settings") fixes, for inverse problems:

* beta = lambda sigma^-2 {1, 4, 8, 16, 32} with
  lambda = min(N^-1 |A^t A|_F^2 |A|_2^-2, 250 sigma^2)  (lambda = 1 for A = I);
* the start x = (A^t A + 0.2 sigma^2 / lambda * Lap)^-1 A^t y.

Readings: A x is the periodic convolution of x with a centred odd-sized
kernel h, (A x)[i, j] = sum_{u,v} h[u, v] x[i - (u - ch), j - (v - cw)]
(indices mod H, W); "the image Laplacian" is the positive semidefinite
periodic 5-point operator (4 x[i,j] minus its four neighbours), whose
Fourier eigenvalues are 4 - 2 cos(2 pi k / H) - 2 cos(2 pi l / W).  Patch
extraction, selection, estimation and reprojection are those of Alg. 1 on
the valid patches (oracle/epll64.py): only the image estimation changes.
"""
from __future__ import annotations

import numpy as np

from . import epll64 as o


def kernel_spectrum(h, H: int, W: int):
    """DFT (H x W, complex) of the centred kernel h embedded with its centre
    at pixel (0, 0): the eigenvalues of A."""
    h = np.asarray(h, dtype=np.float64)
    kh, kw = h.shape
    e = np.zeros((H, W))
    for u in range(kh):
        for v in range(kw):
            e[(u - kh // 2) % H, (v - kw // 2) % W] += h[u, v]
    return np.fft.fft2(e)


def apply_A(x, h):
    """A x (periodic convolution)."""
    Hh = kernel_spectrum(h, *x.shape)
    return np.real(np.fft.ifft2(np.fft.fft2(x) * Hh))


def laplacian_spectrum(H: int, W: int):
    """Fourier eigenvalues of the periodic 5-point Laplacian (PSD sign)."""
    k = np.arange(H)[:, None]
    l = np.arange(W)[None, :]
    return 4.0 - 2.0 * np.cos(2 * np.pi * k / H) - 2.0 * np.cos(2 * np.pi * l / W)


def lambda_param(h, H: int, W: int, sigma: float) -> float:
    """lambda = min(N^-1 |A^t A|_F^2 |A|_2^-2, 250 sigma^2) (Sec. 5): with
    A's eigenvalues a_w, |A^t A|_F^2 = sum |a_w|^4 and |A|_2 = max |a_w|."""
    a2 = np.abs(kernel_spectrum(h, H, W)) ** 2
    return float(min(np.sum(a2 * a2) / (H * W) / a2.max(), 250.0 * sigma * sigma))


def default_betas(h, H, W, sigma):
    return lambda_param(h, H, W, sigma) / sigma ** 2 * np.array([1.0, 4.0, 8.0, 16.0, 32.0])


def initial_estimate(y, h, sigma):
    """x = (A^t A + 0.2 sigma^2 / lambda Lap)^-1 A^t y (Sec. 5)."""
    H, W = y.shape
    Hh = kernel_spectrum(h, H, W)
    lam = lambda_param(h, H, W, sigma)
    den = np.abs(Hh) ** 2 + 0.2 * sigma * sigma / lam * laplacian_spectrum(H, W)
    return np.real(np.fft.ifft2(np.conj(Hh) * np.fft.fft2(y) / den))


def image_update(y, xt, h, beta, sigma):
    """x = (A^t A + beta sigma^2 I)^-1 (A^t y + beta sigma^2 x~) (Alg. 1,
    image estimation), solved in the Fourier basis."""
    H, W = y.shape
    Hh = kernel_spectrum(h, H, W)
    b = beta * sigma * sigma
    X = (np.conj(Hh) * np.fft.fft2(y) + b * np.fft.fft2(xt)) / (np.abs(Hh) ** 2 + b)
    return np.real(np.fft.ifft2(X))


def hqs_iteration(xh, y, h, U, lam, w, sigma, beta):
    """One pass of Alg. 1 with the operator A (patch steps on xh, then the
    image estimation above)."""
    H, W = xh.shape
    r, c = o.patch_corners(H, W)
    _, nu, gamma, L = o.eigen_terms(lam, w, beta)
    Zt, m = o.remove_dc(o.extract(xh, r, c))
    cost = o.selection_costs(Zt, U, nu, L)
    lab, best, second = o.select(cost)
    Zh = o.patch_estimate(Zt, m, lab, U, gamma)
    xt = o.reproject(Zh, H, W)
    return image_update(y, xt, h, beta, sigma), dict(labels=lab, best=best, second=second,
                                                     xtilde=xt)


def restore(y, h, U, lam, w, sigma, betas=None, init=None, trace=False):
    """EPLL deblurring: T iterations of Alg. 1 from the Sec. 5 start (or
    ``init``) over the Sec. 5 schedule (or ``betas``)."""
    y = np.asarray(y, dtype=np.float64)
    H, W = y.shape
    if betas is None:
        betas = default_betas(h, H, W, sigma)
    xh = initial_estimate(y, h, sigma) if init is None else np.asarray(init, np.float64).copy()
    hist = []
    for beta in np.asarray(betas, dtype=np.float64):
        xh, info = hqs_iteration(xh, y, h, U, lam, w, sigma, float(beta))
        if trace:
            info["x"] = xh.copy()
            hist.append(info)
    return (xh, hist) if trace else xh
