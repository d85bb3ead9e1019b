"""Pins of the search-tree reference (oracle/tree.py, Sec. 3.2) and of the
tree builder (paper_1710_08124_amd/tree.py, offline setup)."""
import numpy as np
import pytest

import fepll_synth as fs
from oracle import epll64 as o
from oracle import tree as tr


@pytest.fixture(scope="module")
def small():
    U, lam, w = fs.gmm(12, 21)
    # a hand-made tree: root -> 2 -> 4 -> 12 leaves (3 per node)
    sizes = [1, 2, 4, 12]
    parents = [np.array([0, 0]), np.array([0, 1, 1, 0]),
               np.array([0, 2, 1, 3, 0, 2, 1, 3, 0, 2, 1, 3])]
    return U, lam, w, sizes, parents


def test_root_is_the_mixture_covariance(small):
    U, lam, w, sizes, parents = small
    lev = tr.nodes(U, lam, w, sizes, parents)
    S = np.stack([U[k] @ np.diag(lam[k]) @ U[k].T for k in range(12)])
    np.testing.assert_allclose(lev[0][0], [1.0], rtol=1e-12)
    np.testing.assert_allclose(lev[0][1][0], np.einsum("k,kpq->pq", w, S), rtol=1e-10, atol=1e-9)


def test_nodes_average_their_leaves(small):
    """A node's covariance is the weighted average of all leaves below it
    (moment matching is associative)."""
    U, lam, w, sizes, parents = small
    lev = tr.nodes(U, lam, w, sizes, parents)
    S = np.stack([U[k] @ np.diag(lam[k]) @ U[k].T for k in range(12)])
    leaf_to_l2 = parents[2]
    for node in range(4):
        ks = np.nonzero(leaf_to_l2 == node)[0]
        want = np.einsum("k,kpq->pq", w[ks], S[ks]) / w[ks].sum()
        np.testing.assert_allclose(lev[2][1][node], want, rtol=1e-10, atol=1e-9)
        assert abs(lev[2][0][node] - w[ks].sum()) < 1e-14


def test_flat_tree_is_the_full_search(small):
    """Root with every component as a child: the descent is the argmin of
    Alg. 1 over all K."""
    U, lam, w, _, _ = small
    c = fs.config_c1()
    x = c["y"][:20, :20]
    r, cc = o.patch_corners(20, 20)
    Zt, _ = o.remove_dc(o.extract(x, r, cc))
    beta = 4.0 / 400.0
    lab, _, _ = tr.descend(Zt, U, lam, w, [1, 12], [np.zeros(12, int)], beta)
    _, nu, _, L = o.eigen_terms(lam, w, beta)
    want, _, _ = o.select(o.selection_costs(Zt, U, nu, L))
    np.testing.assert_array_equal(lab, want)


def test_descent_takes_the_best_child_by_slogdet(small):
    """Brute force: at every level the chosen child has the smallest Alg. 1
    cost (explicit covariance, slogdet, solve) among the children."""
    U, lam, w, sizes, parents = small
    x = fs.config_c1()["y"][:12, :12]
    r, cc = o.patch_corners(12, 12)
    Zt, _ = o.remove_dc(o.extract(x, r, cc))
    beta = 2.0 / 400.0
    lab, path, _ = tr.descend(Zt, U, lam, w, sizes, parents, beta)
    lev = tr.nodes(U, lam, w, sizes, parents)
    for i in range(0, Zt.shape[0], 7):
        cur = 0
        for n in range(1, len(sizes)):
            wl, S = lev[n]
            ch = np.nonzero(parents[n - 1] == cur)[0]
            costs = []
            for k in ch:
                M = S[k] + np.eye(64) / beta
                costs.append(-2 * np.log(wl[k]) + np.linalg.slogdet(M)[1]
                             + Zt[i] @ np.linalg.solve(M, Zt[i]))
            cur = ch[int(np.argmin(costs))]
            assert path[i, n - 1] == cur
        assert lab[i] == cur


def test_builder_partitions_are_balanced_and_valid():
    from paper_1710_08124_amd import tree as tb
    U, lam, w = fs.gmm(40, 5)
    sizes, parents = tb.build_tree(U, lam, w, levels=(12, 6, 3, 1))
    assert sizes == [1, 3, 6, 12, 40]
    for n in range(1, len(sizes)):
        p = parents[n - 1]
        assert p.shape == (sizes[n],) and p.min() == 0 and p.max() == sizes[n - 1] - 1
        cnt = np.bincount(p, minlength=sizes[n - 1])
        assert cnt.max() - cnt.min() <= 1  # sizes as equal as the counts allow


def test_builder_beats_random_partitions():
    from paper_1710_08124_amd import tree as tb
    U, lam, w = fs.gmm(48, 6)
    D = tb.sym_kl(tb.covariances(U, lam))
    lab = tb.balanced_partition(D, 16)
    g = np.random.default_rng(1)
    rand = [tb.cluster_cost(D, g.permutation(np.repeat(np.arange(16), 3))) for _ in range(50)]
    assert tb.cluster_cost(D, lab) < min(rand)


def test_builder_kl_matches_definition():
    from paper_1710_08124_amd import tree as tb
    U, lam, w = fs.gmm(4, 7)
    S = tb.covariances(U, lam)
    D = tb.sym_kl(S, eps=0.0)
    for a in range(4):
        for b in range(4):
            want = 0.5 * np.trace(np.linalg.solve(S[b], S[a]) + np.linalg.solve(S[a], S[b])
                                  - 2 * np.eye(64)) if a != b else 0.0
            assert abs(D[a, b] - want) <= 1e-6 * max(1.0, abs(want))
