"""Flat-tail spectrum approximation (Sec. 3.1) -- the reference definition.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
benchmark's CPU-baseline leg may import this module; the restoration library
never does, and this module imports nothing from it.

Sec. 3.1 replaces, in each component, the smallest eigenvalues carrying the
last 1 - rho of the variability by their average: r_k is the smallest rank
whose leading eigenvalues hold at least rho of the trace, and every
eigenvalue after it becomes lambda_k = (sum of the tail) / (P - r_k).  The
restoration is then EPLL with this spectrum, and the paper rewrites its
Gaussian selection and patch estimation so that only the r_k leading
eigenvectors are projected on, plus the squared norm of z~ once per patch:

  cost_k = iota_k + r_k^c log nu_P + |z~|^2 / nu_P
           + sum_{j <= r_k} (log nu_j + c_j^2 / nu_j - c_j^2 / nu_P),
  z^     = U_bar diag(gamma_j - gamma_P) U_bar^t z~ + gamma_P z~  (+ mean),

with c = U_bar^t z~, nu_P = lambda_k + 1/beta, gamma_P = lambda_k / nu_P.
``flat_tail_costs`` and ``flat_tail_estimate`` write these forms out; they
must agree with the plain eigenspace forms of epll64 on the flat-tailed
spectrum (pinned).
"""
from __future__ import annotations

import numpy as np

from . import epll64 as o


def flat_tail(lam, rho: float):
    """(lam_ft, r): the flat-tailed spectra (K x P, eigenvalues decreasing
    per row) and the ranks r_k (1..P).  rho in (0, 1]."""
    lam = np.asarray(lam, dtype=np.float64)
    K, P = lam.shape
    out = lam.copy()
    r = np.empty(K, dtype=np.int64)
    for k in range(K):
        # Sec. 3.1 does not fix a summation order: the trace, the partial
        # sums and the tail sum are taken in index order
        cum = np.cumsum(lam[k])
        total = cum[-1]
        rk = P
        for j in range(P):  # the smallest rank holding rho of the trace
            if cum[j] >= rho * total:
                rk = j + 1
                break
        r[k] = rk
        if rk < P:
            out[k, rk:] = np.cumsum(lam[k, rk:])[-1] / (P - rk)
    return out, r


def flat_tail_costs(Zt, U, lam_ft, r, w, beta):
    """Selection objective (n x K) in the flat-tail form of Sec. 3.1."""
    Zt = np.asarray(Zt, dtype=np.float64)
    n, P = Zt.shape
    K = U.shape[0]
    iota = -2.0 * np.log(np.asarray(w, dtype=np.float64))
    nz2 = np.sum(Zt * Zt, axis=1)
    cost = np.empty((n, K))
    for k in range(K):
        rk = int(r[k])
        nu = lam_ft[k] + 1.0 / beta
        C = Zt @ U[k][:, :rk]
        if rk < P:
            nuP = nu[rk]
            tail = (P - rk) * np.log(nuP) + nz2 / nuP
            inv_p = 1.0 / nuP
        else:  # no tail: the norm term and the correction vanish
            tail = 0.0
            inv_p = 0.0
        cost[:, k] = (iota[k] + tail + np.sum(np.log(nu[:rk]))
                      + (C * C) @ (1.0 / nu[:rk] - inv_p))
    return cost


def flat_tail_estimate(Zt, m, lab, U, lam_ft, r, beta):
    """Patch estimation (n x P) in the flat-tail form of Sec. 3.1."""
    Zt = np.asarray(Zt, dtype=np.float64)
    n, P = Zt.shape
    Zh = np.empty_like(Zt)
    for i in range(n):
        k = int(lab[i])
        rk = int(r[k])
        nu = lam_ft[k] + 1.0 / beta
        gam = lam_ft[k] / nu
        gP = gam[rk] if rk < P else 0.0
        Ub = U[k][:, :rk]
        c = Ub.T @ Zt[i]
        Zh[i] = Ub @ ((gam[:rk] - gP) * c) + gP * Zt[i] + m[i]
    return Zh


def restore(y, U, lam, w, sigma, rho, betas=None, trace=False):
    """EPLL with the flat-tailed mixture (Sec. 3.1), as epll64.restore."""
    lam_ft, _ = flat_tail(lam, rho)
    return o.restore(y, U, lam_ft, w, sigma, betas=betas, trace=trace)
