"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Every check here uses a route to the answer that differs from the oracle's
own: a closed form derived by hand, the dense matrix form of Alg. 1 (explicit
covariances, log-determinants, linear solves, explicit P_i selection
matrices) instead of the eigenspace form, or an invariance of the method.
"""
import numpy as np
import pytest

import fepll_synth as fs
from oracle import epll64 as o

B = np.array([1.0, 4.0, 8.0, 16.0, 32.0])


# ------------------------------------------------------------ helpers

def box_sum(a, h, w):
    """Sum over every h x w window fully inside a (valid mode), by 2-D
    cumulative sums."""
    c = np.zeros((a.shape[0] + 1, a.shape[1] + 1))
    c[1:, 1:] = np.cumsum(np.cumsum(a, 0), 1)
    return c[h:, w:] - c[:-h, w:] - c[h:, :-w] + c[:-h, :-w]


def selection_matrices(H, W, periodic=False):
    """Dense P_i (64 x HW) for every patch, ordered like the oracle."""
    mats = []
    rows = range(H) if periodic else range(H - 7)
    cols = range(W) if periodic else range(W - 7)
    for r in rows:
        for c in cols:
            Pm = np.zeros((64, H * W))
            for dy in range(8):
                for dx in range(8):
                    Pm[8 * dy + dx, ((r + dy) % H) * W + (c + dx) % W] = 1.0
            mats.append(Pm)
    return mats


def dense_iteration(x, y, Sig, w, beta, sigma, periodic=False, closed_form=False):
    """One HQS iteration written in the matrix form of Alg. 1 with dense
    covariances: Gaussian selection by log-determinant and linear solve,
    patch estimation (Sigma + I/beta)^-1 Sigma z~, reprojection with explicit
    P_i matrices.  ``closed_form`` uses Eq. (6) instead of
    the reprojection + image estimation split."""
    H, W = x.shape
    K = Sig.shape[0]
    mats = selection_matrices(H, W, periodic)
    xv = x.ravel()
    num = np.zeros(H * W)
    D = np.zeros(H * W)
    labels = []
    one = np.ones(64) / 64.0
    for Pm in mats:
        z = Pm @ xv
        m = one @ z
        zt = z - m
        costs = []
        for k in range(K):
            Ck = Sig[k] + np.eye(64) / beta
            _, logdet = np.linalg.slogdet(Ck)
            costs.append(-2 * np.log(w[k]) + logdet + zt @ np.linalg.solve(Ck, zt))
        k = int(np.argmin(costs))
        labels.append(k)
        zh = np.linalg.solve(Sig[k] + np.eye(64) / beta, Sig[k] @ zt) + m
        num += Pm.T @ zh
        D += Pm.T @ np.ones(64)
    b = beta * sigma ** 2
    if closed_form:
        Pn = 64.0
        xn = (y.ravel() + (b / Pn) * num) / (1.0 + (b / Pn) * D)
    else:
        xn = (y.ravel() + b * (num / D)) / (1.0 + b)
    return xn.reshape(H, W), np.array(labels)


def covs(U, lam):
    return np.einsum("kij,kj,klj->kil", U, lam, U)


# ------------------------------------------------------------------ P1

@pytest.mark.parametrize("shape", [(12, 12), (17, 23)])
def test_p1_isotropic_single_component(shape):
    """K=1, Sigma = s I: patch estimation is the scalar shrink
    m + s/(s + 1/beta) (z - m); the reprojection is then
    g x + (1-g) * (average of the covering patch means)."""
    H, W = shape
    g = fs.rng(5)
    y = g.uniform(0, 255, (H, W))
    s = 37.0
    U = np.eye(64)[None]
    lam = np.full((1, 64), s)
    w = np.array([1.0])
    sigma = 15.0
    betas = B / sigma ** 2
    got = o.restore(y, U, lam, w, sigma)
    x = y.copy()
    # covering counts and covering sums of means by box sums over the
    # zero-padded grid of patch corners
    for beta in betas:
        gfac = s / (s + 1.0 / beta)
        means = box_sum(x, 8, 8) / 64.0          # (H-7, W-7)
        pad = np.zeros((H + 7, W + 7))
        pad[7:H, 7:W] = means
        msum = box_sum(pad, 8, 8)               # sum of covering means
        one = np.zeros((H + 7, W + 7))
        one[7:H, 7:W] = 1.0
        cnt = box_sum(one, 8, 8)
        xt = gfac * x + (1 - gfac) * msum / cnt
        b = beta * sigma ** 2
        x = (y + b * xt) / (1 + b)
    np.testing.assert_allclose(got, x, rtol=0, atol=1e-10)


# ------------------------------------------------------------------ P2

def test_p2_single_component_dense_operator():
    """K=1 general Sigma on a 12x12 image: every iteration is the linear map
    x -> (y + b M x)/(1 + b), M = D^-1 sum_i P_i^t W P_i,
    W = (Sigma + I/beta)^-1 Sigma (I - 11^t/64) + 11^t/64."""
    H = W = 12
    U, lam, _ = fs.gmm(1, 7)
    w = np.array([1.0])
    Sig = covs(U, lam)[0]
    g = fs.rng(8)
    y = g.uniform(0, 255, (H, W))
    sigma = 20.0
    mats = selection_matrices(H, W)
    D = sum(Pm.T @ np.ones(64) for Pm in mats)
    x = y.ravel().copy()
    J = np.ones((64, 64)) / 64.0
    for beta in B / sigma ** 2:
        Wf = np.linalg.solve(Sig + np.eye(64) / beta, Sig) @ (np.eye(64) - J) + J
        M = sum(Pm.T @ Wf @ Pm for Pm in mats) / D[:, None]
        b = beta * sigma ** 2
        x = (y.ravel() + b * (M @ x)) / (1 + b)
    got = o.restore(y, U, lam, w, sigma)
    np.testing.assert_allclose(got.ravel(), x, rtol=0, atol=1e-9)


# ------------------------------------------------------------------ P3

def test_p3_single_patch_textbook_wiener():
    """8x8 image: one patch, one iteration is (y + b W y)/(1 + b) with the
    component picked by the dense Gaussian likelihood."""
    U, lam, w = fs.gmm(3, 9)
    Sig = covs(U, lam)
    g = fs.rng(10)
    y = g.uniform(0, 255, (8, 8))
    sigma = 25.0
    beta = 1.0 / sigma ** 2
    z = y.ravel()
    zt = z - z.mean()
    cost = [-2 * np.log(w[k]) + np.linalg.slogdet(Sig[k] + np.eye(64) / beta)[1]
            + zt @ np.linalg.solve(Sig[k] + np.eye(64) / beta, zt) for k in range(3)]
    k = int(np.argmin(cost))
    zh = np.linalg.solve(Sig[k] + np.eye(64) / beta, Sig[k] @ zt) + z.mean()
    want = (z + zh) / 2.0  # b = beta sigma^2 = 1
    got, info = o.hqs_iteration(y, y, U, lam, w, sigma, beta, want_costs=True)
    assert info["labels"][0] == k
    np.testing.assert_allclose(info["costs"][0], cost, rtol=1e-11)
    np.testing.assert_allclose(got.ravel(), want, rtol=0, atol=1e-10)


# ------------------------------------------------------------------ P4

@pytest.mark.parametrize("K,seed", [(2, 1), (3, 2), (4, 3)])
def test_p4_bruteforce_selection_tiny_K(K, seed):
    """Full dense iteration (matrix form of Alg. 1) on a 11x13 image equals
    the oracle's eigenspace iteration: labels identical, image to 1e-9."""
    U, lam, w = fs.gmm(K, seed)
    Sig = covs(U, lam)
    g = fs.rng(seed + 100)
    y = fs.dead_leaves(11, 13, seed + 50) + g.normal(0, 20, (11, 13))
    x = y + g.normal(0, 3, y.shape)
    sigma = 20.0
    for beta in (1 / 400.0, 16 / 400.0):
        want, wl = dense_iteration(x, y, Sig, w, beta, sigma)
        got, info = o.hqs_iteration(x, y, U, lam, w, sigma, beta)
        np.testing.assert_array_equal(info["labels"], wl)
        np.testing.assert_allclose(got, want, rtol=0, atol=1e-9)


def test_p4_bruteforce_costs_c1():
    """K=20 (the 64x64 workload's mixture): selection costs of a sample of
    patches by log-determinant + solve agree to 1e-9 relative, same argmin,
    and best/second are the two smallest costs."""
    c = fs.config_c1()
    U, lam, w, y = c["U"], c["lam"], c["w"], c["y"]
    Sig = covs(U, lam)
    sigma = c["sigma"]
    beta = 4.0 / sigma ** 2
    _, info = o.hqs_iteration(y, y, U, lam, w, sigma, beta, want_costs=True)
    r, cc = o.patch_corners(64, 64)
    g = fs.rng(3)
    for i in g.choice(r.size, 40, replace=False):
        z = y[r[i]:r[i] + 8, cc[i]:cc[i] + 8].ravel()
        zt = z - z.mean()
        cost = np.array([-2 * np.log(w[k]) + np.linalg.slogdet(Sig[k] + np.eye(64) / beta)[1]
                         + zt @ np.linalg.solve(Sig[k] + np.eye(64) / beta, zt)
                         for k in range(20)])
        np.testing.assert_allclose(info["costs"][i], cost, rtol=1e-9)
        assert info["labels"][i] == int(np.argmin(cost))
        srt = np.sort(cost)
        np.testing.assert_allclose([info["best"][i], info["second"][i]], srt[:2], rtol=1e-9)


# ------------------------------------------------------------------ P5

@pytest.mark.parametrize("H,W", [(8, 8), (9, 20), (64, 64), (31, 17)])
def test_p5_counts_closed_form(H, W):
    """Aggregating all-ones patches gives cnt(r, c) = cr(r) cc(c) with
    cr(r) = min(r, H-8) - max(0, r-7) + 1; sum = 64 N_p; interior 64."""
    Np = (H - 7) * (W - 7)
    S, cnt = o.aggregate(np.ones((Np, 64)), H, W)
    cr = np.array([min(r, H - 8) - max(0, r - 7) + 1 for r in range(H)], float)
    cc = np.array([min(c, W - 8) - max(0, c - 7) + 1 for c in range(W)], float)
    np.testing.assert_array_equal(cnt, np.outer(cr, cc))
    np.testing.assert_array_equal(S, cnt)
    assert cnt.sum() == 64 * Np
    if H >= 15 and W >= 15:
        assert np.all(cnt[7:H - 7, 7:W - 7] == 64)


# ------------------------------------------------------------------ P6

def test_p6_periodic_equals_closed_form():
    """With wrap-around patches every pixel is covered P = 64 times and
    Alg. 1 (average, then image estimation) equals the closed-form x-update
    Eq. (6); both are computed densely here, and the oracle's
    periodic iteration must match."""
    U, lam, w = fs.gmm(3, 4)
    Sig = covs(U, lam)
    g = fs.rng(44)
    H, W = 9, 10
    y = g.uniform(0, 255, (H, W))
    x = y + g.normal(0, 5, (H, W))
    sigma, beta = 20.0, 8.0 / 400.0
    a, la = dense_iteration(x, y, Sig, w, beta, sigma, periodic=True)
    b, lb = dense_iteration(x, y, Sig, w, beta, sigma, periodic=True, closed_form=True)
    np.testing.assert_array_equal(la, lb)
    np.testing.assert_allclose(a, b, rtol=0, atol=1e-10)
    got, info = o.hqs_iteration(x, y, U, lam, w, sigma, beta, periodic=True)
    np.testing.assert_array_equal(info["labels"], la)
    np.testing.assert_allclose(got, a, rtol=0, atol=1e-9)


def test_p6_valid_mode_differs_only_on_border():
    """Valid patches: Alg. 1 and Eq. (6) agree where the
    count is P and differ on the border band (the reading taken: Alg. 1)."""
    U, lam, w = fs.gmm(2, 6)
    Sig = covs(U, lam)
    g = fs.rng(45)
    H = W = 17
    y = g.uniform(0, 255, (H, W))
    sigma, beta = 20.0, 4.0 / 400.0
    a, _ = dense_iteration(y, y, Sig, w, beta, sigma)
    b, _ = dense_iteration(y, y, Sig, w, beta, sigma, closed_form=True)
    np.testing.assert_allclose(a[7:10, 7:10], b[7:10, 7:10], atol=1e-10)
    assert np.abs(a - b).max() > 1e-3
    got = o.hqs_iteration(y, y, U, lam, w, sigma, beta)[0]
    np.testing.assert_allclose(got, a, atol=1e-9)


# ------------------------------------------------------------------ P7

def test_p7_identity_as_sigma_vanishes():
    """sigma -> 0: 1/beta -> 0, gamma -> 1 and x_hat -> y with
    ||x_hat - y||_inf proportional to sigma^2."""
    c = fs.config_c1()
    U, lam, w = c["U"], c["lam"], c["w"]
    y = c["x"][:24, :24]
    errs = []
    for s in (1e-2, 1e-3, 1e-4):
        xh = o.restore(y, U, lam, w, s)
        errs.append(np.abs(xh - y).max() / s ** 2)
    assert errs[0] > 0
    for e in errs[1:]:
        assert abs(e / errs[0] - 1.0) < 0.05, errs


# ------------------------------------------------------------------ P8

def test_p8_flat_prior_returns_input():
    U, _, _ = fs.gmm(3, 13)
    lam = np.full((3, 64), 1e12)
    w = np.array([0.2, 0.3, 0.5])
    y = fs.rng(1).uniform(0, 255, (20, 20))
    xh = o.restore(y, U, lam, w, 10.0)
    np.testing.assert_allclose(xh, y, rtol=0, atol=1e-6)


# ------------------------------------------------------------------ P9

@pytest.fixture(scope="module")
def small():
    U, lam, w = fs.gmm(6, 21)
    x = fs.test_image(24, 28, 77)
    y = fs.noisy(x, 20.0, 78)
    ref, hist = o.restore(y, U, lam, w, 20.0, trace=True)
    return U, lam, w, y, ref, hist


def test_p9_shift_invariance(small):
    U, lam, w, y, ref, hist = small
    got, h2 = o.restore(y + 13.25, U, lam, w, 20.0, trace=True)
    np.testing.assert_allclose(got, ref + 13.25, atol=1e-9)
    for a, b in zip(hist, h2):
        np.testing.assert_array_equal(a["labels"], b["labels"])


def test_p9_scale_invariance(small):
    """x(s y; s sigma, s^2 lambda) = s x(y; sigma, lambda): every cost moves
    by the same 64 log s^2, so the labels do not change."""
    U, lam, w, y, ref, hist = small
    s = 3.0
    got, h2 = o.restore(s * y, U, s * s * lam, w, 20.0 * s, trace=True)
    np.testing.assert_allclose(got, s * ref, atol=1e-8)
    for a, b in zip(hist, h2):
        np.testing.assert_array_equal(a["labels"], b["labels"])
        np.testing.assert_allclose(b["best"] - a["best"], 64 * np.log(s * s), atol=1e-8)


def test_p9_eigenvector_sign_flips(small):
    U, lam, w, y, ref, hist = small
    sgn = np.where(fs.rng(2).random((U.shape[0], 64)) < 0.5, -1.0, 1.0)
    got = o.restore(y, U * sgn[:, None, :], lam, w, 20.0)
    np.testing.assert_allclose(got, ref, atol=1e-9)


def test_p9_component_permutation(small):
    U, lam, w, y, ref, hist = small
    perm = fs.rng(3).permutation(U.shape[0])
    got, h2 = o.restore(y, U[perm], lam[perm], w[perm], 20.0, trace=True)
    np.testing.assert_allclose(got, ref, atol=1e-9)
    inv = np.argsort(perm)
    for a, b in zip(hist, h2):
        np.testing.assert_array_equal(perm[b["labels"]], a["labels"])


def test_p9_duplicate_component_lowest_index(small):
    """Appending a copy of component 0 (weights renormalised, so every cost
    moves by the same constant) ties it with 0 exactly: 0 must win."""
    U, lam, w, y, ref, hist = small
    U2 = np.concatenate([U, U[:1]])
    lam2 = np.concatenate([lam, lam[:1]])
    w2 = np.concatenate([w, w[:1]]) / (1.0 + w[0])
    got, h2 = o.restore(y, U2, lam2, w2, 20.0, trace=True)
    np.testing.assert_allclose(got, ref, atol=1e-9)
    for a, b in zip(hist, h2):
        np.testing.assert_array_equal(a["labels"], b["labels"])
        assert np.all(b["labels"] < U.shape[0])


def test_p9_vanishing_weight_component(small):
    U, lam, w, y, ref, hist = small
    U2 = np.concatenate([U, U[2:3]])
    lam2 = np.concatenate([lam, lam[2:3]])
    w2 = np.concatenate([w, [1e-300]])
    got = o.restore(y, U2, lam2, w2, 20.0)
    np.testing.assert_allclose(got, ref, atol=1e-9)


def test_second_best_is_second_smallest(small):
    U, lam, w, y, ref, hist = small
    _, info = o.hqs_iteration(y, y, U, lam, w, 20.0, 1 / 400.0, want_costs=True)
    srt = np.sort(info["costs"], axis=1)
    np.testing.assert_array_equal(info["best"], srt[:, 0])
    np.testing.assert_array_equal(info["second"], srt[:, 1])
