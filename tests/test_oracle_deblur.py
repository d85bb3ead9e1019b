"""Pins of the deblurring reference (oracle/deblur.py): every Fourier-domain
formula against the dense-matrix definition on tiny images, and the
identity operator against plain denoising."""
import numpy as np
import pytest

import fepll_synth as fs
from oracle import deblur as db
from oracle import epll64 as o


def dense_A(h, H, W):
    """A as an explicit N x N matrix from the convolution sum."""
    N = H * W
    A = np.zeros((N, N))
    kh, kw = h.shape
    for i in range(H):
        for j in range(W):
            for u in range(kh):
                for v in range(kw):
                    A[i * W + j, ((i - (u - kh // 2)) % H) * W + (j - (v - kw // 2)) % W] += h[u, v]
    return A


def dense_lap(H, W):
    N = H * W
    L = np.zeros((N, N))
    for i in range(H):
        for j in range(W):
            p = i * W + j
            L[p, p] += 4.0
            for di, dj in ((1, 0), (-1, 0), (0, 1), (0, -1)):
                L[p, ((i + di) % H) * W + (j + dj) % W] -= 1.0
    return L


@pytest.fixture
def small():
    H, W = 10, 12
    g = np.random.default_rng(3)
    h = fs.blur_kernel(5, 9)
    return H, W, h, g


def test_convolution_matches_dense(small):
    H, W, h, g = small
    x = g.standard_normal((H, W))
    np.testing.assert_allclose(db.apply_A(x, h).ravel(), dense_A(h, H, W) @ x.ravel(),
                               atol=1e-12)


def test_lambda_matches_dense_norms(small):
    H, W, h, _ = small
    A = dense_A(h, H, W)
    AtA = A.T @ A
    want = min(np.sum(AtA * AtA) / (H * W) / np.linalg.norm(A, 2) ** 2, 250 * 0.5 ** 2)
    assert abs(db.lambda_param(h, H, W, 0.5) - want) < 1e-12 * max(1, want)
    # the 250 sigma^2 cap binds for small sigma
    assert db.lambda_param(h, H, W, 0.01) == pytest.approx(250 * 0.01 ** 2)
    # identity: lambda = 1
    assert db.lambda_param(np.ones((1, 1)), H, W, 5.0) == pytest.approx(1.0, abs=1e-14)


def test_laplacian_spectrum_matches_dense(small):
    H, W, _, g = small
    x = g.standard_normal((H, W))
    got = np.real(np.fft.ifft2(np.fft.fft2(x) * db.laplacian_spectrum(H, W))).ravel()
    np.testing.assert_allclose(got, dense_lap(H, W) @ x.ravel(), atol=1e-12)


def test_init_and_update_solve_the_dense_systems(small):
    H, W, h, g = small
    y = g.standard_normal((H, W)) * 30 + 100
    xt = g.standard_normal((H, W)) * 30 + 100
    sigma, beta = 0.5, 3.0
    A = dense_A(h, H, W)
    lam = db.lambda_param(h, H, W, sigma)
    M = A.T @ A + 0.2 * sigma ** 2 / lam * dense_lap(H, W)
    np.testing.assert_allclose(db.initial_estimate(y, h, sigma).ravel(),
                               np.linalg.solve(M, A.T @ y.ravel()), rtol=1e-9, atol=1e-8)
    b = beta * sigma ** 2
    want = np.linalg.solve(A.T @ A + b * np.eye(H * W), A.T @ y.ravel() + b * xt.ravel())
    np.testing.assert_allclose(db.image_update(y, xt, h, beta, sigma).ravel(), want,
                               rtol=1e-10, atol=1e-9)


def test_identity_operator_is_denoising():
    """A = I with the denoising start x = y and schedule: the deblurring
    iteration is Alg. 1's denoising iteration."""
    c = fs.config_c1()
    y = c["y"][:30, :34]
    want = o.restore(y, c["U"], c["lam"], c["w"], c["sigma"])
    got = db.restore(y, np.ones((1, 1)), c["U"], c["lam"], c["w"], c["sigma"],
                     betas=o.default_betas(c["sigma"]), init=y)
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-9)
    # and the Sec. 5 schedule reduces to the denoising one
    np.testing.assert_allclose(db.default_betas(np.ones((1, 1)), 30, 34, c["sigma"]),
                               o.default_betas(c["sigma"]), rtol=1e-14)


def test_blur_kernel_and_degradation():
    h = fs.blur_kernel(9, 801)
    assert h.shape == (9, 9) and abs(h.sum() - 1) < 1e-12 and h.min() >= 0
    x = fs.test_image(20, 24, 5)
    y0 = fs.blurred(x, h, 0.0, 1)
    np.testing.assert_allclose(y0, db.apply_A(x, h), atol=1e-9)
