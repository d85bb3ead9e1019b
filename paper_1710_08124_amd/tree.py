"""Balanced Gaussian search tree for the selection step (Sec. 3.2): offline
construction on the host (float64 NumPy), for GMM.set_tree.

Sec. 3.2 collapses the mixture level by level (K = 200 -> 64 -> 32 -> 16 ->
8 -> 4 -> 2 -> 1 components), each level a partition of the one below into
clusters of about equal size minimizing the summed symmetric Kullback-Leibler
divergence between the zero-mean Gaussians of a cluster (the clustering cost of Sec. 3.2,
whose printed form compares a component with itself: the pairwise
divergence is meant).  The paper solves each partition with a genetic
algorithm for the multiple travelling salesmen problem; here a deterministic
solver of the same objective with the cluster sizes fixed (as equal as the
counts allow): a greedy fill (seed = the free component farthest from the
others, then its nearest free components), then pairwise swaps between
clusters while any lowers the total.  The moment-matched merge of a cluster
(weights summed, covariances averaged with the weights) gives the next
level; the library performs the same merge for the node tables.
"""
from __future__ import annotations

import numpy as np

LEVELS_K200 = (64, 32, 16, 8, 4, 2, 1)


def covariances(U, lam):
    U = np.asarray(U, np.float64)
    lam = np.asarray(lam, np.float64)
    return np.einsum("kpj,kj,kqj->kpq", U, lam, U)


def sym_kl(S, eps: float = 1e-6):
    """Pairwise symmetric KL divergences of zero-mean Gaussians with
    covariances S (K x P x P): 0.5 tr(S2^-1 S1 + S1^-1 S2 - 2 I).  A small
    ridge (eps times the mean trace / P) keeps singular covariances
    invertible."""
    S = np.asarray(S, np.float64)
    K, P, _ = S.shape
    ridge = eps * np.trace(S, axis1=1, axis2=2).mean() / P
    R = S + ridge * np.eye(P)[None]
    inv = np.linalg.inv(R)
    # tr(inv_b R_a) for all a, b
    T = np.einsum("bpq,aqp->ab", inv, R)
    D = 0.5 * (T + T.T) - P
    np.fill_diagonal(D, 0.0)
    return np.maximum(D, 0.0)


def _sizes(K: int, L: int):
    q, r = divmod(K, L)
    return [q + 1] * r + [q] * (L - r)


def balanced_partition(D, L: int, max_passes: int = 50):
    """Partition of range(K) into L clusters of sizes as equal as possible,
    approximately minimizing the summed within-cluster divergence D."""
    K = D.shape[0]
    sizes = _sizes(K, L)
    free = np.ones(K, bool)
    label = np.full(K, -1, np.int64)
    for l, sz in enumerate(sizes):
        idx = np.nonzero(free)[0]
        far = idx[np.argmax(D[np.ix_(idx, idx)].sum(1))]  # ties: lowest index
        members = [far]
        free[far] = False
        while len(members) < sz:
            idx = np.nonzero(free)[0]
            cost = D[np.ix_(idx, members)].sum(1)
            nxt = idx[np.argmin(cost)]
            members.append(nxt)
            free[nxt] = False
        label[members] = l
    # swap refinement: exchange two components of different clusters while
    # the total within-cluster divergence decreases
    for _ in range(max_passes):
        improved = False
        for a in range(K):
            la = label[a]
            ca = D[a, label == la].sum()
            best, arg = 0.0, -1
            for b in range(K):
                lb = label[b]
                if lb == la:
                    continue
                cb = D[b, label == lb].sum()
                # a moves to lb (without b), b moves to la (without a)
                new = (D[a, label == lb].sum() - D[a, b]) + (D[b, label == la].sum() - D[b, a])
                delta = new - (ca + cb)
                if delta < best - 1e-12:
                    best, arg = delta, b
            if arg >= 0:
                label[a], label[arg] = label[arg], label[a]
                improved = True
        if not improved:
            break
    return label


def cluster_cost(D, label):
    total = 0.0
    for l in np.unique(label):
        m = np.nonzero(label == l)[0]
        total += D[np.ix_(m, m)].sum() / 2
    return total


def merge(w, S, label):
    """Moment-matched merge of zero-mean Gaussians: per cluster, the summed
    weight and the weight-averaged covariance."""
    L = int(label.max()) + 1
    wn = np.zeros(L)
    Sn = np.zeros((L,) + S.shape[1:])
    for k in range(len(w)):
        wn[label[k]] += w[k]
        Sn[label[k]] += w[k] * S[k]
    return wn, Sn / wn[:, None, None]


def build_tree(U, lam, w, levels=LEVELS_K200):
    """Level sizes (root first: 1, ..., K) and the parent arrays (one per
    level below the root: parents[n][i] is the node of level n - 1 that
    node i of level n belongs to), built from the leaves up."""
    S = covariances(U, lam)
    w = np.asarray(w, np.float64)
    K = S.shape[0]
    sizes = [K]
    parents = []
    for L in levels:
        if L >= sizes[-1]:
            raise ValueError("levels must shrink")
        label = balanced_partition(sym_kl(S), L)
        parents.append(label.astype(np.int32))
        w, S = merge(w, S, label)
        sizes.append(L)
    if sizes[-1] != 1:
        raise ValueError("the last level must have one node")
    return sizes[::-1], parents[::-1]
