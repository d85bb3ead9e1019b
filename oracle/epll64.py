"""Plain FP64 CPU EPLL denoising -- the oracle.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
benchmark's CPU-baseline leg may import this module; the restoration library
never does, and this module imports nothing from it.

What it computes (Parameswaran, Deledalle, Denis, Nguyen, "Accelerating
GMM-based patch priors for image restoration", arXiv 1710.08124):

* the EPLL MAP problem with a zero-mean GMM patch prior on DC-removed 8x8
  patches (Sec. 2, Eq. (1) and Eq. (2));
* approximated by half-quadratic splitting (Eq. (3)) with the five
  steps of Algorithm 1 -- patch extraction, Gaussian selection, patch
  estimation, patch reprojection, image estimation -- for denoising (A = I);
* the selection and estimation steps written in each component's eigenbasis
  (Sec. 2.1, Eqs. (7) and (8)
  and the two lines after them), with iota_k = -2 log w_k,
  nu_kj = S_kjj + 1/beta and gamma_kj = S_kjj / nu_kj;
* the schedule T = 5, beta = {1, 4, 8, 16, 32} / sigma^2 and the start
  x = y (end of Sec. 2 "Algorithm"; lambda = 1 for denoising, Sec. 5
  "Parameter settings").

Readings taken where the paper is silent (each one is listed in the design
notes with its reason):

* patch set: every 8x8 patch fully inside the image, indexed by its top-left
  pixel (r, c), 0 <= r <= H-8, 0 <= c <= W-8, in row-major order of (r, c);
  the reprojection divides by the actual number of covering patches
  (Alg. 1, patch reprojection).  ``periodic=True`` instead takes one patch at
  every pixel with wrap-around, so that every pixel is covered P = 64 times.
* patch vector: z[8*dy + dx] = x[r + dy, c + dx];
* DC: the patch mean m is removed before selection and shrinkage and added
  back unshrunk after patch estimation;
* ties in the selection go to the lowest component index;
* the score reported per patch is the selection objective of Alg. 1
  (iota_k + sum_j log nu_kj + c_j^2 / nu_kj), in "cost" units; a margin in
  nats is half a cost difference.

Everything is float64; matrix products go through NumPy (BLAS).  Patches are
processed in blocks of ``block`` rows only to bound memory: blocking changes
no arithmetic.
"""
from __future__ import annotations

import numpy as np

P = 64
PS = 8
DEFAULT_B = (1.0, 4.0, 8.0, 16.0, 32.0)


# --------------------------------------------------------------- schedule

def default_betas(sigma: float) -> np.ndarray:
    """beta_t = {1, 4, 8, 16, 32} / sigma^2 (Sec. 2, after Alg. 1)."""
    return np.asarray(DEFAULT_B, dtype=np.float64) / (float(sigma) ** 2)


# ---------------------------------------------------- patch extraction

def patch_corners(H: int, W: int, periodic: bool = False):
    """Top-left corners (r, c) of the patch set, row-major in (r, c)."""
    if periodic:
        rr, cc = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    else:
        rr, cc = np.meshgrid(np.arange(H - PS + 1), np.arange(W - PS + 1), indexing="ij")
    return rr.ravel(), cc.ravel()


def extract(x: np.ndarray, r: np.ndarray, c: np.ndarray, periodic: bool = False):
    """Patch extraction z_i = P_i x (Alg. 1, first step) -> (n, 64)."""
    H, W = x.shape
    Z = np.empty((r.size, P))
    for dy in range(PS):
        for dx in range(PS):
            rr = r + dy
            cc = c + dx
            if periodic:
                rr = rr % H
                cc = cc % W
            Z[:, PS * dy + dx] = x[rr, cc]
    return Z


def remove_dc(Z: np.ndarray):
    """Split each patch into its mean and the zero-mean part (Sec. 2: the
    GMM prior models patches with their DC component removed)."""
    m = Z.mean(axis=1)
    return Z - m[:, None], m


# ------------------------------------------------------ per-beta terms

def eigen_terms(lam: np.ndarray, w: np.ndarray, beta: float):
    """iota_k, nu_kj, gamma_kj of the eigenspace formulation and the
    per-component constant L_k = iota_k + sum_j log nu_kj."""
    nu = lam + 1.0 / beta
    iota = -2.0 * np.log(w)
    gamma = lam / nu
    L = iota + np.log(nu).sum(axis=1)
    return iota, nu, gamma, L


# --------------------------------------------------- Gaussian selection

def selection_costs(Zt: np.ndarray, U: np.ndarray, nu: np.ndarray, L: np.ndarray):
    """Selection objective of every component for every patch, (n, K):
    c^k = U_k^t z~ (Eq. (7)) and
    cost_k = iota_k + sum_j (log nu_kj + c_j^2 / nu_kj)
    (Eq. (8))."""
    n = Zt.shape[0]
    K = U.shape[0]
    cost = np.empty((n, K))
    for k in range(K):
        C = Zt @ U[k]                  # row i holds (U_k^t z~_i)^t
        cost[:, k] = L[k] + (C * C) @ (1.0 / nu[k])
    return cost


def select(cost: np.ndarray):
    """k* = argmin_k cost (lowest index on ties), the best and the second
    smallest cost of each patch."""
    lab = np.argmin(cost, axis=1)
    best = cost[np.arange(cost.shape[0]), lab]
    if cost.shape[1] > 1:
        two = np.partition(cost, 1, axis=1)
        second = two[:, 1]
    else:
        second = np.full(cost.shape[0], np.inf)
    return lab, best, second


# ---------------------------------------------------- patch estimation

def patch_estimate(Zt: np.ndarray, m: np.ndarray, lab: np.ndarray, U: np.ndarray,
                   gamma: np.ndarray):
    """Wiener estimate in the chosen eigenbasis:
    c = U_k*^t z~, c_hat = gamma_k* * c, z_hat = U_k* c_hat, plus the
    patch mean added back (eigenspace form of Alg. 1, patch estimation)."""
    Zh = np.empty_like(Zt)
    for k in np.unique(lab):
        sel = np.nonzero(lab == k)[0]
        C = Zt[sel] @ U[k]
        Zh[sel] = (C * gamma[k][None, :]) @ U[k].T
    return Zh + m[:, None]


# ------------------------------------------------- patch reprojection

def aggregate(Zh: np.ndarray, H: int, W: int, periodic: bool = False):
    """Sum_i P_i^t z_i and the diagonal of Sum_i P_i^t P_i (patch counts),
    for the full patch set of ``patch_corners`` (rows of Zh in that order).
    Entry 8*dy + dx of patch (r, c) lands on pixel (r + dy, c + dx)."""
    S = np.zeros((H, W))
    cnt = np.zeros((H, W))
    if periodic:
        for dy in range(PS):
            for dx in range(PS):
                plane = Zh[:, PS * dy + dx].reshape(H, W)
                S += np.roll(plane, (dy, dx), axis=(0, 1))
                cnt += 1.0
        return S, cnt
    Hp, Wp = H - PS + 1, W - PS + 1
    for dy in range(PS):
        for dx in range(PS):
            S[dy:dy + Hp, dx:dx + Wp] += Zh[:, PS * dy + dx].reshape(Hp, Wp)
            cnt[dy:dy + Hp, dx:dx + Wp] += 1.0
    return S, cnt


def reproject(Zh, H, W, periodic=False):
    """x~ = (Sum P_i^t P_i)^-1 Sum P_i^t z_hat_i (Alg. 1, patch
    reprojection): the average of the overlapping restored patches."""
    S, cnt = aggregate(Zh, H, W, periodic)
    return S / cnt


# --------------------------------------------------- image estimation

def image_update(y: np.ndarray, xt: np.ndarray, beta: float, sigma: float):
    """x = (A^t A + beta sigma^2 I)^-1 (A^t y + beta sigma^2 x~) with A = I
    (Alg. 1, image estimation)."""
    b = beta * sigma * sigma
    return (y + b * xt) / (1.0 + b)


# -------------------------------------------------------- one iteration

def hqs_iteration(xh, y, U, lam, w, sigma, beta, periodic=False, block=4096,
                  want_costs=False):
    """One pass of Alg. 1 from the current estimate ``xh``.

    Returns (x_new, info) with info = dict(labels, best, second[, costs]).
    """
    H, W = xh.shape
    r, c = patch_corners(H, W, periodic)
    _, nu, gamma, L = eigen_terms(lam, w, beta)
    n = r.size
    lab = np.empty(n, dtype=np.int64)
    best = np.empty(n)
    second = np.empty(n)
    Zh = np.empty((n, P))
    costs = np.empty((n, U.shape[0])) if want_costs else None
    for s in range(0, n, block):
        e = min(n, s + block)
        Z = extract(xh, r[s:e], c[s:e], periodic)
        Zt, m = remove_dc(Z)
        cost = selection_costs(Zt, U, nu, L)
        lab[s:e], best[s:e], second[s:e] = select(cost)
        if want_costs:
            costs[s:e] = cost
        Zh[s:e] = patch_estimate(Zt, m, lab[s:e], U, gamma)
    xt = reproject(Zh, H, W, periodic)
    x_new = image_update(y, xt, beta, sigma)
    info = dict(labels=lab, best=best, second=second, xtilde=xt)
    if want_costs:
        info["costs"] = costs
    return x_new, info


def restore(y, U, lam, w, sigma, betas=None, init=None, periodic=False,
            block=4096, trace=False, want_costs=False):
    """EPLL denoising by HQS: T iterations of Alg. 1 from x = y (or
    ``init``) over the beta schedule (default {1,4,8,16,32}/sigma^2).

    Returns x_hat, or (x_hat, per-iteration list of dict(x, labels, best,
    second[, costs])) when ``trace`` is set.
    """
    y = np.asarray(y, dtype=np.float64)
    if betas is None:
        betas = default_betas(sigma)
    xh = y.copy() if init is None else np.asarray(init, dtype=np.float64).copy()
    hist = []
    for beta in np.asarray(betas, dtype=np.float64):
        xh, info = hqs_iteration(xh, y, U, lam, w, sigma, float(beta), periodic,
                                 block, want_costs)
        if trace:
            info["x"] = xh.copy()
            hist.append(info)
    return (xh, hist) if trace else xh


# ------------------------------------------------------------ helpers

def patch_scores(z: np.ndarray, U, lam, w, beta):
    """Selection objective of all K components for a handful of raw
    (not DC-removed) patches z, shape (n, 64) -> (n, K)."""
    Zt, _ = remove_dc(np.atleast_2d(np.asarray(z, dtype=np.float64)))
    _, nu, _, L = eigen_terms(lam, w, beta)
    return selection_costs(Zt, U, nu, L)


def psnr(x_ref: np.ndarray, x: np.ndarray) -> float:
    """10 log10(255^2 / MSE) over all pixels, no clipping."""
    mse = float(np.mean((np.asarray(x, np.float64) - np.asarray(x_ref, np.float64)) ** 2))
    return 10.0 * np.log10(255.0 ** 2 / mse)
