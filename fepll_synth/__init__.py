"""Seeded synthetic inputs for the EPLL restoration path.

This module draws the inputs that both the FP64 oracle and the HIP path
consume: a synthetic zero-mean Gaussian mixture (eigenbases, eigenvalues,
weights), dead-leaves images, 1/f Gaussian texture, white Gaussian noise and
the uneven batch of images.  It holds none of the restoration arithmetic
(no patch extraction, scoring, shrinkage, aggregation or image update), so
that the oracle and the GPU path share nothing but their inputs.

Random streams: NumPy ``Generator(PCG64(seed))``.  Recipes:

* GMM (stands in for the trained K=200, 8x8 patch mixture the paper uses in
  its parameter settings): for each component an orthogonal U_k from the QR
  factorisation of a standard normal 64x64 matrix, with the signs fixed so
  that diag(R) > 0 (Haar distributed); eigenvalues 2000 * j^-2 * U[0.5, 2]
  drawn independently per (k, j), j = 1..64, then sorted in decreasing order
  (the eigendecomposition the paper assumes orders them that way);
  weights from a flat Dirichlet(1).
* Dead leaves: disks with centres uniform on the canvas enlarged by r_max on
  every side, radius density proportional to r^-3 on [1, min(H, W)/2]
  (inverse-CDF draw), grey level U[0, 255]; disks are laid front to back and
  a disk only paints pixels no earlier disk covers, until every pixel is
  covered.
* 1/f texture: white N(0, 1) field, multiplied by 1/|f| in the Fourier domain
  with the DC coefficient set to zero, real part, rescaled to a given std.
* Noise: x + sigma * N(0, 1), no clipping, no quantisation (sigma is the
  standard deviation on the [0, 255] scale, as in the paper's observation
  model y = A x + w with A = I).
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "rng", "gmm", "dead_leaves", "texture_1f", "noisy", "test_image",
    "config_c1", "config_c2", "config_c3", "batch_c5", "training_images",
    "mlp_init",
]


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def gmm(K: int, seed: int, d: int = 64):
    """Synthetic zero-mean GMM as (U, lam, w).

    U:   (K, d, d) float64, column j of U[k] is the j-th eigenvector of
         Sigma_k, pixel index 8*dy + dx (row-major 8x8 patch).
    lam: (K, d) float64, eigenvalues of Sigma_k in decreasing order.
    w:   (K,) float64, positive, summing to one.
    """
    g = rng(seed)
    U = np.empty((K, d, d))
    lam = np.empty((K, d))
    j = np.arange(1, d + 1, dtype=np.float64)
    for k in range(K):
        A = g.standard_normal((d, d))
        Q, R = np.linalg.qr(A)
        s = np.sign(np.diag(R))
        s[s == 0] = 1.0
        U[k] = Q * s[None, :]
        lam[k] = np.sort(2000.0 * j ** -2 * g.uniform(0.5, 2.0, d))[::-1]
    w = g.dirichlet(np.ones(K))
    return U, lam, w


def _paint_small(img, cov, cy, cx, r, v):
    """Paint a batch of small disks front to back onto uncovered pixels."""
    H, W = img.shape
    R = int(np.ceil(r.max()))
    off = np.arange(-R, R + 1)
    oy, ox = np.meshgrid(off, off, indexing="ij")
    oy = oy.ravel()
    ox = ox.ravel()
    iy = np.floor(cy).astype(np.int64)[:, None] + oy[None, :]
    ix = np.floor(cx).astype(np.int64)[:, None] + ox[None, :]
    inside = ((iy - cy[:, None]) ** 2 + (ix - cx[:, None]) ** 2 <= (r ** 2)[:, None])
    inside &= (iy >= 0) & (iy < H) & (ix >= 0) & (ix < W)
    di, _ = np.nonzero(inside)
    if di.size == 0:
        return
    pix = iy[inside] * W + ix[inside]
    free = ~cov.ravel()[pix]
    di = di[free]
    pix = pix[free]
    if pix.size == 0:
        return
    # entries are already ordered by disk index (row-major nonzero), so the
    # first occurrence of a pixel is the front-most disk covering it
    upix, first = np.unique(pix, return_index=True)
    img.ravel()[upix] = v[di[first]]
    cov.ravel()[upix] = True


def dead_leaves(H: int, W: int, seed: int, g: np.random.Generator | None = None):
    """Dead-leaves image, float64 in [0, 255], shape (H, W)."""
    if g is None:
        g = rng(seed)
    img = np.zeros((H, W))
    cov = np.zeros((H, W), dtype=bool)
    rmax = min(H, W) / 2.0
    batch = 65536
    n = 0
    while not cov.all():
        u = g.random(batch)
        r = (1.0 - u * (1.0 - rmax ** -2)) ** -0.5
        cy = g.uniform(-rmax, H + rmax, batch)
        cx = g.uniform(-rmax, W + rmax, batch)
        v = g.uniform(0.0, 255.0, batch)
        # keep disks that can touch the canvas
        keep = (cy + r >= 0) & (cy - r <= H - 1) & (cx + r >= 0) & (cx - r <= W - 1)
        idx = np.nonzero(keep)[0]
        # walk the batch in order; big disks one by one, small ones in runs
        i = 0
        while i < idx.size:
            j = i
            while j < idx.size and j - i < 8192 and r[idx[j]] <= 6.0:
                j += 1
            if j > i:
                sel = idx[i:j]
                _paint_small(img, cov, cy[sel], cx[sel], r[sel], v[sel])
                i = j
                continue
            t = idx[i]
            y0 = max(0, int(np.floor(cy[t] - r[t])))
            y1 = min(H, int(np.ceil(cy[t] + r[t])) + 1)
            x0 = max(0, int(np.floor(cx[t] - r[t])))
            x1 = min(W, int(np.ceil(cx[t] + r[t])) + 1)
            yy, xx = np.ogrid[y0:y1, x0:x1]
            m = ((yy - cy[t]) ** 2 + (xx - cx[t]) ** 2 <= r[t] ** 2) & ~cov[y0:y1, x0:x1]
            img[y0:y1, x0:x1][m] = v[t]
            cov[y0:y1, x0:x1] |= m
            i += 1
        n += batch
    return img


def texture_1f(H: int, W: int, std: float, seed: int | None = None,
               g: np.random.Generator | None = None):
    """Zero-mean Gaussian texture with a 1/|f| amplitude spectrum."""
    if g is None:
        g = rng(seed)
    white = g.standard_normal((H, W))
    fy = np.fft.fftfreq(H)[:, None]
    fx = np.fft.fftfreq(W)[None, :]
    f = np.sqrt(fy ** 2 + fx ** 2)
    filt = np.zeros_like(f)
    nz = f > 0
    filt[nz] = 1.0 / f[nz]
    t = np.real(np.fft.ifft2(np.fft.fft2(white) * filt))
    t -= t.mean()
    return t * (std / t.std())


def noisy(x: np.ndarray, sigma: float, seed: int):
    g = rng(seed)
    return x + sigma * g.standard_normal(x.shape)


def test_image(H: int, W: int, seed: int, texture_std: float = 10.0):
    """Dead leaves plus 1/f texture of the given std (0 disables it)."""
    g = rng(seed)
    x = dead_leaves(H, W, seed, g=g)
    if texture_std > 0:
        x = x + texture_1f(H, W, texture_std, g=g)
    return x


# ---------------------------------------------------------------- workloads

def config_c1():
    """64x64 dead leaves, sigma 20, K=20 GMM (seed 11)."""
    x = dead_leaves(64, 64, 101)
    y = noisy(x, 20.0, 201)
    U, lam, w = gmm(20, 11)
    return dict(x=x, y=y, sigma=20.0, U=U, lam=lam, w=w)


def config_c2(sigma: float, size: int = 512):
    """Dead leaves + 1/f texture (std 10), K=200 GMM (seed 12)."""
    seeds = {10.0: 202, 25.0: 203, 50.0: 204}
    x = test_image(size, size, 102)
    y = noisy(x, sigma, seeds.get(float(sigma), 202))
    U, lam, w = gmm(200, 12)
    return dict(x=x, y=y, sigma=float(sigma), U=U, lam=lam, w=w)


def config_c3(size: int = 1024):
    """size^2 dead leaves + 1/f texture, sigma 25, K=200 GMM (seed 12)."""
    x = test_image(size, size, 103)
    y = noisy(x, 25.0, 205)
    U, lam, w = gmm(200, 12)
    return dict(x=x, y=y, sigma=25.0, U=U, lam=lam, w=w)


def _c5_item(args):
    H, W, img_seed, noise_seed, sig, texture_std = args
    x = test_image(H, W, img_seed, texture_std)
    return dict(x=x, y=noisy(x, sig, noise_seed), sigma=sig)


def batch_c5(n: int = 48, seed: int = 500, texture_std: float = 10.0, workers: int = 1):
    """Uneven batch: image 0 is 256x256, image n-1 is 1024 rows x 1536 cols,
    the rest H ~ U{256..1024}, W ~ U{256..1536}; sigma ~ U[5, 50].

    workers > 1 draws the images in that many forked processes (same
    images: each has its own seeds); fork only from a process that has not
    initialised a GPU."""
    g = rng(seed)
    shapes = [(256, 256)]
    for _ in range(n - 2):
        shapes.append((int(g.integers(256, 1025)), int(g.integers(256, 1537))))
    shapes.append((1024, 1536))
    sig = g.uniform(5.0, 50.0, n)
    img_seeds = g.integers(1, 2 ** 31 - 1, n)
    noise_seeds = g.integers(1, 2 ** 31 - 1, n)
    items = [(H, W, int(img_seeds[i]), int(noise_seeds[i]), float(sig[i]), texture_std)
             for i, (H, W) in enumerate(shapes[:n])]
    if workers <= 1:
        return [_c5_item(a) for a in items]
    import multiprocessing as mp
    with mp.get_context("fork").Pool(workers) as pool:
        return pool.map(_c5_item, items, chunksize=1)


def training_images(seeds=range(300, 313), size: int = 256, sigma_seed: int = 600,
                    sigmas: str = "uniform"):
    """Clean/noisy pairs for the proposal network's training set.

    sigmas: how image i of n draws its noise level (one uniform draw u_i of
    the sigma_seed stream per image, in order):
    * "uniform": sigma ~ U[5, 50];
    * "low": the first n // 2 images log-uniform over [4.5, 10], the others
      over [10, 50], each half stratified (image j of m takes
      a (b / a)^((j + u_i) / m) on its interval [a, b]).  The network's
      recall is lowest where sigma is small (sharper posteriors), so half the
      data sits there."""
    g = rng(sigma_seed)
    out = []
    seeds = list(seeds)
    n = len(seeds)
    h = n // 2
    for i, s in enumerate(seeds):
        u = float(g.uniform(0.0, 1.0)) if sigmas == "low" else None
        if sigmas == "low":
            a0, a1, j, m = (4.5, 10.0, i, h) if i < h else (10.0, 50.0, i - h, n - h)
            sig = a0 * (a1 / a0) ** ((j + u) / m)
        elif sigmas == "uniform":
            sig = float(g.uniform(5.0, 50.0))
        else:
            raise ValueError(f"unknown sigma schedule {sigmas!r}")
        x = test_image(size, size, s)
        out.append(dict(x=x, y=noisy(x, sig, s + 1000), sigma=sig))
    return out


def mlp_init(K: int = 200, seed: int = 700, d_in: int = 65, hidden: int = 256):
    """Initial weights of the proposal network, float64:
    W ~ U(-1/sqrt(fan_in), 1/sqrt(fan_in)), b = 0; W stored (out, in)."""
    g = rng(seed)
    dims = [(hidden, d_in), (hidden, hidden), (K, hidden)]
    p = {}
    for i, (o, n) in enumerate(dims, start=1):
        a = 1.0 / np.sqrt(n)
        p[f"W{i}"] = g.uniform(-a, a, (o, n))
        p[f"b{i}"] = np.zeros(o)
    return p


# ----------------------------------------------------------- deblurring

def blur_kernel(size: int = 9, seed: int = 800, steps: int = 60):
    """A seeded motion-blur-like kernel (size x size, odd, centred, sums to
    1): the visits of a random walk with momentum started at the centre,
    smoothed by a 3-tap binomial filter.  Stands in for the blur kernel of
    the paper's deblurring experiments, which is not available here."""
    if size % 2 == 0:
        raise ValueError("size must be odd")
    g = rng(seed)
    k = np.zeros((size, size))
    c = size // 2
    p = np.array([float(c), float(c)])
    v = g.normal(size=2)
    v /= np.linalg.norm(v)
    for _ in range(steps):
        v = 0.8 * v + 0.45 * g.normal(size=2)
        v /= max(np.linalg.norm(v), 1e-9)
        p = np.clip(p + 0.5 * v, 0, size - 1)
        k[int(round(p[0])), int(round(p[1]))] += 1.0
    b = np.array([0.25, 0.5, 0.25])
    k = np.apply_along_axis(lambda r: np.convolve(r, b, mode="same"), 0, k)
    k = np.apply_along_axis(lambda r: np.convolve(r, b, mode="same"), 1, k)
    return k / k.sum()


def blurred(x: np.ndarray, h: np.ndarray, sigma: float, seed: int):
    """y = h (*) x + n: periodic convolution of x with the centred kernel h
    (entry (u, v) of h weighs x[i - (u - c), j - (v - c)]), then Gaussian
    noise of std sigma (seeded)."""
    H, W = x.shape
    kh, kw = h.shape
    e = np.zeros((H, W))
    for u in range(kh):
        for v in range(kw):
            e[(u - kh // 2) % H, (v - kw // 2) % W] += h[u, v]
    y = np.real(np.fft.ifft2(np.fft.fft2(x) * np.fft.fft2(e)))
    return y + sigma * rng(seed).standard_normal((H, W))


def config_deblur(size: int = 512, sigma: float = 0.5, ksize: int = 9):
    """The deblurring workload: the size^2 test image blurred by a 9x9
    seeded motion kernel, noise sigma 0.5 (the paper's deblurring noise
    level), K = 200 GMM (seed 12)."""
    x = test_image(size, size, 104)
    h = blur_kernel(ksize, 801)
    y = blurred(x, h, sigma, 206)
    U, lam, w = gmm(200, 12)
    return dict(x=x, y=y, h=h, sigma=sigma, U=U, lam=lam, w=w)
