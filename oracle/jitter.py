"""Jittered stochastic patch subsampling (Sec. 3.3) -- the reference definition.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
benchmark's CPU-baseline leg may import this module; the restoration library
never does, and this module imports nothing from it.

Sec. 3.3 runs every iteration of Alg. 1 on a random subset of the patches:
the points of a grid of spacing s (in both directions), shifted as a whole
by a random offset, each point moved independently and uniformly by at most
floor((sqrt(P) - s) / 2) pixels per direction, resampled at every iteration,
so that every pixel is covered by at least one patch.  Selection and patch
estimation run on the subset only, and the reprojection averages the
subset's overlapping restored patches.

The paper leaves the random source and the grid's extent open.  Reading:

* random numbers: Philox4x32-10 (Salmon, Moraes, Dror and Shaw, "Parallel
  random numbers: as easy as 1, 2, 3", SC 2011), key = the 64-bit seed
  (low word, high word).  Grid point (a, c) of iteration t uses counter
  (t, a, c, 0): output word 0 moves its row, word 1 its column; the global
  shift uses counter (t, 0xffffffff, 0xffffffff, 0): word 0 for rows, word
  1 for columns.  A uniform integer in {0..n-1} is the word modulo n
  (n <= 8: bias below 2^-29).
* grid: b = floor((8 - s) / 2); shift g uniform in {0..s-1}; grid rows
  i0 = g - s n0 + s a for a = 0, 1, ..., where n0 is the smallest n with
  g - s n <= -b, up to the first a with i0 - b >= Hp - 1 (Hp = H - 7
  patch rows); the same for columns.  A point's patch starts at
  clamp(i0 + d, 0, Hp - 1) with d uniform in {-b..b}.  Consecutive starts
  then differ by at most s + 2 b <= 8 and the first and last are clamped to
  0 and Hp - 1: every pixel is covered.  The subset is the set of distinct
  patches (clamping may bring two points together).
"""
from __future__ import annotations

import numpy as np

from . import epll64 as o

_M0 = np.uint64(0xD2511F53)
_M1 = np.uint64(0xCD9E8D57)
_W0 = np.uint64(0x9E3779B9)
_W1 = np.uint64(0xBB67AE85)
_MASK = np.uint64(0xFFFFFFFF)


def philox4x32_10(counter, key):
    """Philox4x32 with 10 rounds on arrays of counters (..., 4) and a key
    (2,) of uint32; returns (..., 4) uint32.

    One round: with (hi0, lo0) = M0 * c0 and (hi1, lo1) = M1 * c2 (64-bit
    products split into high and low words), the new counter is
    (hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0); between rounds the key is
    bumped by the Weyl constants (k0 + W0, k1 + W1) mod 2^32."""
    c = np.asarray(counter, dtype=np.uint64) & _MASK
    k0 = np.uint64(int(key[0]) & 0xFFFFFFFF)
    k1 = np.uint64(int(key[1]) & 0xFFFFFFFF)
    c0, c1, c2, c3 = c[..., 0], c[..., 1], c[..., 2], c[..., 3]
    for rnd in range(10):
        p0 = _M0 * c0
        p1 = _M1 * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & _MASK
        hi1, lo1 = p1 >> np.uint64(32), p1 & _MASK
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
        if rnd < 9:
            k0 = (k0 + _W0) & _MASK
            k1 = (k1 + _W1) & _MASK
    return np.stack([c0, c1, c2, c3], axis=-1).astype(np.uint32)


def _seed_key(seed: int):
    seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    return (seed & 0xFFFFFFFF, seed >> 32)


def grid_axis(n_patch: int, s: int, g: int):
    """Grid coordinates i0 along one axis with n_patch patch starts."""
    b = (8 - s) // 2
    n0 = -((-(g + b)) // s)  # ceil((g + b) / s): g - s n0 <= -b
    first = g - s * n0
    out = []
    i0 = first
    while True:
        out.append(i0)
        if i0 - b >= n_patch - 1:
            break
        i0 += s
    return np.asarray(out, dtype=np.int64)


def positions(H: int, W: int, s: int, seed: int, t: int):
    """Sorted flat indices r * Wp + c of the distinct patches of iteration t
    (Wp = W - 7), and the grid (rows, cols, per-point starts) for pins."""
    if not 1 <= s <= 8:
        raise ValueError("s must be in 1..8")
    Hp, Wp = H - 7, W - 7
    key = _seed_key(seed)
    b = (8 - s) // 2
    sh = philox4x32_10(np.array([t, 0xFFFFFFFF, 0xFFFFFFFF, 0], np.uint64), key)
    gy, gx = int(sh[0]) % s, int(sh[1]) % s
    rows = grid_axis(Hp, s, gy)
    cols = grid_axis(Wp, s, gx)
    a, c = np.meshgrid(np.arange(rows.size), np.arange(cols.size), indexing="ij")
    ctr = np.stack([np.full(a.shape, t), a, c, np.zeros(a.shape, np.int64)], axis=-1)
    u = philox4x32_10(ctr.astype(np.uint64), key).astype(np.int64)
    dy = u[..., 0] % (2 * b + 1) - b
    dx = u[..., 1] % (2 * b + 1) - b
    r = np.clip(rows[a] + dy, 0, Hp - 1)
    cc = np.clip(cols[c] + dx, 0, Wp - 1)
    idx = np.unique((r * Wp + cc).ravel())
    return idx, dict(rows=rows, cols=cols, r=r, c=cc, gy=gy, gx=gx)


def hqs_iteration(xh, y, U, lam, w, sigma, beta, idx):
    """One pass of Alg. 1 over the patch subset idx (flat indices r Wp + c):
    selection and estimation of those patches, then the average of their
    overlapping estimates (every pixel covered) and the image update."""
    xt, info = subset_estimate(xh, U, lam, w, beta, idx)
    return o.image_update(y, xt, beta, sigma), info


def subset_estimate(xh, U, lam, w, beta, idx):
    """The patch steps of Alg. 1 on the subset idx: selection and estimation
    of those patches and the average x~ of their overlapping estimates
    (every pixel covered), before any image estimation."""
    H, W = xh.shape
    Wp = W - 7
    r, c = np.divmod(np.asarray(idx, dtype=np.int64), Wp)
    _, nu, gamma, L = o.eigen_terms(lam, w, beta)
    Zt, m = o.remove_dc(o.extract(xh, r, c))
    cost = o.selection_costs(Zt, U, nu, L)
    lab, best, second = o.select(cost)
    Zh = o.patch_estimate(Zt, m, lab, U, gamma)
    S = np.zeros((H, W))
    cnt = np.zeros((H, W))
    for i in range(r.size):
        S[r[i]:r[i] + 8, c[i]:c[i] + 8] += Zh[i].reshape(8, 8)
        cnt[r[i]:r[i] + 8, c[i]:c[i] + 8] += 1.0
    if np.any(cnt == 0):
        raise AssertionError("a pixel is not covered by the subset")
    return S / cnt, dict(labels=lab, best=best, second=second, idx=np.asarray(idx), count=cnt)


def restore(y, U, lam, w, sigma, s, seed, betas=None, init=None, trace=False):
    """EPLL denoising with jittered subsampling: T iterations, iteration t
    on positions(H, W, s, seed, t)."""
    y = np.asarray(y, dtype=np.float64)
    if betas is None:
        betas = o.default_betas(sigma)
    xh = y.copy() if init is None else np.asarray(init, dtype=np.float64).copy()
    H, W = y.shape
    hist = []
    for t, beta in enumerate(np.asarray(betas, dtype=np.float64)):
        idx, _ = positions(H, W, s, seed, t)
        xh, info = hqs_iteration(xh, y, U, lam, w, sigma, float(beta), idx)
        if trace:
            info["x"] = xh.copy()
            hist.append(info)
    return (xh, hist) if trace else xh
