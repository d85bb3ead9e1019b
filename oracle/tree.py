"""Gaussian selection by a balanced search tree (Sec. 3.2) -- the reference
definition.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
benchmark's CPU-baseline leg may import this module; the restoration library
never does, and this module imports nothing from it.

The tree is given by its level sizes (root first: 1, ..., K) and, for every
level below the root, the parent of each node in the level above.  Its
nodes are zero-mean Gaussians obtained from the leaves (the mixture's
components) by moment matching, level by level upwards: a node's weight is
the sum of its children's, its covariance their weight-averaged covariance.
A patch is compared with the children of the root, follows the child of
smallest selection cost, and so on down to a leaf (ties to the lower
index), the leaf being its label.  The selection cost of a node is Alg. 1's,
in the eigenspace form of Sec. 2.1, with the node's weight, eigenvectors and
eigenvalues.  Optionally every node's spectrum is flat-tailed (Sec. 3.1;
in the paper the flat tail applies to every node of the tree, inner nodes
included).
"""
from __future__ import annotations

import numpy as np

from . import epll64 as o
from . import flat_tail as ft


def nodes(U, lam, w, sizes, parents):
    """Per level (root first) the nodes' weights (n,) and covariances
    (n, P, P): the leaves from (U, lam, w), the levels above by moment
    matching."""
    U = np.asarray(U, np.float64)
    lam = np.asarray(lam, np.float64)
    S = np.stack([U[k] @ np.diag(lam[k]) @ U[k].T for k in range(U.shape[0])])
    wl = np.asarray(w, np.float64)
    out = [(wl, S)]
    for n in range(len(sizes) - 1, 0, -1):
        par = np.asarray(parents[n - 1])
        L = sizes[n - 1]
        wn = np.zeros(L)
        Sn = np.zeros((L,) + S.shape[1:])
        for i in range(par.size):
            wn[par[i]] += wl[i]
            Sn[par[i]] += wl[i] * S[i]
        for l in range(L):
            Sn[l] /= wn[l]
        wl, S = wn, Sn
        out.append((wl, S))
    return out[::-1]


def node_eig(S):
    """Eigenvectors (columns) and eigenvalues, decreasing, clamped at 0."""
    lam, V = np.linalg.eigh(S)
    lam, V = lam[..., ::-1], V[..., ::-1]
    return V, np.maximum(lam, 0.0)


def descend(Zt, U, lam, w, sizes, parents, beta, rho=None):
    """Tree selection for DC-removed patches Zt (n x P).  Returns the leaf
    labels, the path (n x levels, the node chosen at each level below the
    root) and, per level, half the cost gap between the best and the second
    child (inf for a single child)."""
    levels = nodes(U, lam, w, sizes, parents)
    terms = []
    for wl, S in levels:
        V, lm = node_eig(S)
        if rho is not None and rho < 1.0:
            lm, _ = ft.flat_tail(lm, rho)
        _, nu, _, L = o.eigen_terms(lm, wl, beta)
        terms.append((V, nu, L))
    n = Zt.shape[0]
    cur = np.zeros(n, np.int64)  # the root
    path = np.zeros((n, len(sizes) - 1), np.int64)
    gaps = np.zeros((n, len(sizes) - 1))
    for lev in range(1, len(sizes)):
        par = np.asarray(parents[lev - 1])
        V, nu, L = terms[lev]
        cost = o.selection_costs(Zt, V, nu, L)  # every node of the level
        for i in range(n):
            ch = np.nonzero(par == cur[i])[0]  # ascending
            c = cost[i, ch]
            j = int(np.argmin(c))
            srt = np.sort(c)
            gaps[i, lev - 1] = 0.5 * (srt[1] - srt[0]) if c.size > 1 else np.inf
            cur[i] = ch[j]
        path[:, lev - 1] = cur
    return cur, path, gaps


def hqs_iteration(xh, y, U, lam, w, sigma, beta, sizes, parents, rho=None):
    """Alg. 1 with the tree selection; patch estimation with the chosen
    leaf's Wiener filter (on the leaves' spectra, flat-tailed with rho)."""
    H, W = xh.shape
    r, c = o.patch_corners(H, W)
    Zt, m = o.remove_dc(o.extract(xh, r, c))
    lab, path, gaps = descend(Zt, U, lam, w, sizes, parents, beta, rho)
    lam_l = lam if rho is None or rho >= 1.0 else ft.flat_tail(lam, rho)[0]
    _, _, gamma, _ = o.eigen_terms(lam_l, w, beta)
    Zh = o.patch_estimate(Zt, m, lab, U, gamma)
    xt = o.reproject(Zh, H, W)
    return o.image_update(y, xt, beta, sigma), dict(labels=lab, path=path, gaps=gaps)


def restore(y, U, lam, w, sigma, sizes, parents, rho=None, betas=None, trace=False):
    y = np.asarray(y, np.float64)
    if betas is None:
        betas = o.default_betas(sigma)
    x = y.copy()
    hist = []
    for beta in np.asarray(betas, np.float64):
        x, info = hqs_iteration(x, y, U, lam, w, sigma, float(beta), sizes, parents, rho)
        if trace:
            info["x"] = x.copy()
            hist.append(info)
    return (x, hist) if trace else x
