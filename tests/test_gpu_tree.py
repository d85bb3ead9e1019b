"""Gaussian selection by the search tree (Sec. 3.2) on the GPU.

* degenerate trees reproduce the bfloat16 full search bit for bit: a root
  with every component as a child, and the same under a chain of
  single-child nodes, plain and flat-tailed (the node costs are the all-K
  selection's arithmetic);
* on a balanced K = 200 tree, the descent against the FP64 reference
  (oracle/tree.py): labels differ only where the reference's path has, at
  some level, a cost gap within the bfloat16 rounding bound of that level's
  costs;
* restoration through the tree within 0.05 dB of the FP64 tree
  restoration; a batch equals its images restored one by one;
* malformed trees and unsupported option mixes rejected."""
import numpy as np
import pytest

import fepll_synth as fs
from oracle import epll64 as o
from oracle import tree as otree

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def F():
    import paper_1710_08124_amd as F
    F.lib()
    return F


@pytest.fixture(scope="module")
def k200():
    from paper_1710_08124_amd import tree as btree
    c = fs.config_c2(25.0)
    sizes, parents = btree.build_tree(c["U"], c["lam"], c["w"])
    return c, sizes, parents


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def f32(a):
    return np.asarray(a, np.float32).astype(np.float64)


@pytest.mark.parametrize("rho", [None, 0.95])
@pytest.mark.parametrize("chain", [False, True])
def test_degenerate_trees_are_the_full_search(F, rho, chain):
    U, lam, w = fs.gmm(8, 31)
    c = fs.config_c2(25.0)
    x = dev(c["y"][200:296, 100:230])  # several tiles, ragged tail
    beta = float(o.default_betas(25.0)[1])
    g = F.GMM(U, lam, w)
    if rho is not None:
        g.flat_tail(rho)
    lab0, best0, sec0, _ = F.select(g, x, beta, precision="bf16")
    if chain:
        g.set_tree([1, 1, 1, 8], [np.zeros(1), np.zeros(1), np.zeros(8)])
    else:
        g.set_tree([1, 8], [np.zeros(8)])
    lab, best, sec, flags = F.select(g, x, beta, precision="bf16", tree=True)
    assert torch.equal(lab, lab0)
    assert torch.equal(best, best0)
    assert torch.equal(sec, sec0)
    assert not flags.any()


def _level_bounds(Zt, V, nu, L, eps=1.02 * 2.0 ** -7):
    """Bound (n, nodes) on |bfloat16 cost - exact cost| of a level: both
    operands of c_j = sum_p z_p U_pj / sqrt(nu_j) rounded to bfloat16
    (relative 2^-8 each, products exact), so |c_j' - c_j| <= d_j = eps
    sum_p |z_p U_pj| / sqrt(nu_j) and the sum of squares moves by at most
    sum_j 2 |c_j| d_j + d_j^2; float32 sums and the float32 L_k add at most
    70 u (sum_j c_j^2 + |L_k|), u = 2^-24 (the 64-term accumulations with
    the slack of the projection bound)."""
    n = Zt.shape[0]
    out = np.empty((n, V.shape[0]))
    A = np.abs(Zt)
    for k in range(V.shape[0]):
        s = 1.0 / np.sqrt(nu[k])
        C = (Zt @ V[k]) * s
        d = eps * (A @ np.abs(V[k])) * s
        out[:, k] = (np.sum(2 * np.abs(C) * d + d * d, axis=1)
                     + 70 * 2.0 ** -24 * (np.sum(C * C, axis=1) + abs(L[k])))
    return out


def _near_tie_check(c, sizes, parents, beta, Zt, lab):
    """Labels lab of patches Zt against the FP64 descent: every mismatch
    leaves the reference's path at a level whose two compared costs are
    within the bfloat16 bound of each other.  Returns (agreement, all ok)."""
    want, path, gaps = otree.descend(Zt, c["U"], c["lam"], c["w"], sizes, parents, beta)
    agree = float(np.mean(lab == want))
    bad = np.nonzero(lab != want)[0]
    ok = np.zeros(bad.size, bool)
    if bad.size:
        # the GPU's path, from its leaf up (a leaf has one path)
        nl = len(sizes) - 1
        gpath = np.zeros((bad.size, nl), np.int64)
        gpath[:, nl - 1] = lab[bad]
        for lev in range(nl - 1, 0, -1):
            gpath[:, lev - 1] = np.asarray(parents[lev])[gpath[:, lev]]
        # first level where it leaves the reference's path: there the two
        # siblings' costs, each within the bound, must be a near-tie
        first = np.argmax(gpath != path[bad], axis=1)
        levels = otree.nodes(c["U"], c["lam"], c["w"], sizes, parents)
        for lev in range(1, len(sizes)):
            sel = np.nonzero(first == lev - 1)[0]
            if sel.size == 0:
                continue
            wl, S = levels[lev]
            V, lm = otree.node_eig(S)
            _, nu, _, Lk = o.eigen_terms(lm, wl, beta)
            Bl = _level_bounds(Zt[bad[sel]], V, nu, Lk)
            rows = np.arange(sel.size)
            B = np.maximum(Bl[rows, path[bad[sel], lev - 1]], Bl[rows, gpath[sel, lev - 1]])
            # the reference's half gap between best and second child is at
            # most half the gap to the GPU's child: a flip needs it <= B
            ok[sel] = gaps[bad[sel], lev - 1] <= B
    return agree, bad.size, bool(ok.all())


@pytest.mark.parametrize("t", [0, 3])
def test_descent_against_fp64_tree(F, k200, t):
    c, sizes, parents = k200
    x = f32(c["y"][150:246, 90:220])
    beta = float(o.default_betas(25.0)[t])
    g = F.GMM(c["U"], c["lam"], c["w"])
    g.set_tree(sizes, parents)
    lab, _, _, _ = F.select(g, dev(x), beta, precision="bf16", tree=True)
    lab = lab.cpu().numpy()
    H, W = x.shape
    r, cc = o.patch_corners(H, W)
    Zt, _ = o.remove_dc(o.extract(x, r, cc))
    agree, nbad, ok = _near_tie_check(c, sizes, parents, beta, Zt, lab)
    print(f"tree descent t={t}: agreement with FP64 {agree:.5f}, mismatches {nbad}, "
          f"all at near-ties {ok}")
    assert ok
    assert agree >= 0.9  # (the all-K bfloat16 selection's floor; the bound decides)


def test_descent_full_size_sampled(F, k200):
    """The benchmarked configuration: 1024^2, K = 200, sigma 25, first
    iteration; the labels of 2000 sampled patches against the FP64 descent."""
    c, sizes, parents = k200
    c3 = fs.config_c3()
    y32 = f32(c3["y"])
    beta = float(o.default_betas(25.0)[0])
    g = F.GMM(c["U"], c["lam"], c["w"])
    g.set_tree(sizes, parents)
    lab, _, _, _ = F.select(g, dev(y32), beta, precision="bf16", tree=True)
    lab = lab.cpu().numpy()
    Wp = 1024 - 7
    idx = np.sort(fs.rng(4).choice(Wp * Wp, 2000, replace=False))
    Zt, _ = o.remove_dc(o.extract(y32, idx // Wp, idx % Wp))
    agree, nbad, ok = _near_tie_check(c, sizes, parents, beta, Zt, lab[idx])
    print(f"tree 1024^2 sampled: agreement {agree:.5f}, mismatches {nbad}, all at near-ties {ok}")
    assert ok
    assert agree >= 0.9


def test_restoration_quality(F, k200):
    c, sizes, parents = k200
    x0, y = c["x"][128:256, 192:320], f32(c["y"][128:256, 192:320])
    ref = otree.restore(y, c["U"], c["lam"], c["w"], 25.0, sizes, parents)
    full = o.restore(y, c["U"], c["lam"], c["w"], 25.0)
    g = F.GMM(c["U"], c["lam"], c["w"])
    g.set_tree(sizes, parents)
    got = F.restore(g, dev(y), 25.0, precision="bf16", tree=True).cpu().numpy()
    d = o.psnr(x0, ref) - o.psnr(x0, got.astype(np.float64))
    print(f"tree bf16 vs FP64 tree: dPSNR {d:+.4f} dB; FP64 tree vs FP64 full search "
          f"{o.psnr(x0, ref) - o.psnr(x0, full):+.4f} dB (PSNR {o.psnr(x0, ref):.2f})")
    assert abs(d) <= 0.05


def test_flat_tail_tree_quality(F, k200):
    c, sizes, parents = k200
    x0, y = c["x"][128:256, 192:320], f32(c["y"][128:256, 192:320])
    ref = otree.restore(y, c["U"], c["lam"], c["w"], 25.0, sizes, parents, rho=0.95)
    g = F.GMM(c["U"], c["lam"], c["w"])
    g.set_tree(sizes, parents)
    g.flat_tail(0.95)  # after the tree: the tree's spectra follow
    got = F.restore(g, dev(y), 25.0, precision="bf16", tree=True).cpu().numpy()
    d = o.psnr(x0, ref) - o.psnr(x0, got.astype(np.float64))
    print(f"flat tree bf16 vs FP64 flat tree: dPSNR {d:+.4f} dB")
    assert abs(d) <= 0.05


def test_batch_equals_single_images(F, k200):
    c, sizes, parents = k200
    g = F.GMM(c["U"], c["lam"], c["w"])
    g.set_tree(sizes, parents)
    ys = [dev(c["y"][:80, :100]), dev(c["y"][100:164, 50:250]), dev(c["y"][300:309, 0:40])]
    sig = [25.0, 10.0, 50.0]
    outs = F.restore_batch(g, ys, sig, precision="bf16", tree=True)
    for y, s, out in zip(ys, sig, outs):
        one = F.restore(g, y, s, precision="bf16", tree=True)
        assert torch.equal(out, one)


def test_bad_trees_rejected(F):
    U, lam, w = fs.gmm(8, 31)
    g = F.GMM(U, lam, w)
    x = dev(fs.config_c1()["y"][:32, :32])
    with pytest.raises(F.FepllError, match="EINVAL"):
        F.select(g, x, 0.01, precision="bf16", tree=True)  # no tree set
    L = F.lib()
    cases = [
        ([2, 8], [0, 0, 0, 0, 1, 1, 1, 1], -1),  # two roots
        ([1, 7], [0] * 7, -1),  # the leaves are not the K components
        ([1, 2, 8], [0, 0] + [0, 0, 0, 0, 1, 1, 1, 2], -1),  # parent out of its level
        ([1, 2, 8], [0, 0] + [0] * 8, -1),  # node 1 of level 1 without a child
        ([1, 1, 8], [0] + [0] * 8, 0),  # a chain: fine
    ]
    for sizes, par, want in cases:
        s = np.asarray(sizes, np.int32)
        p = np.asarray(par, np.int32)
        st = L.fepll_gmm_set_tree(g.handle, s.size, s.ctypes.data, p.ctypes.data)
        assert st == want, (sizes, par, st)
    U9, lam9, w9 = fs.gmm(9, 32)
    g9 = F.GMM(U9, lam9, w9)
    with pytest.raises(F.FepllError, match="EINVAL"):
        g9.set_tree([1, 9], [np.zeros(9)])  # nine children
    g.set_tree([1, 8], [np.zeros(8)])
    with pytest.raises(F.FepllError, match="EUNSUPPORTED"):
        F.select(g, x, 0.01, precision="fp32", tree=True)
    with pytest.raises(F.FepllError, match="EUNSUPPORTED"):
        F.restore(g, x, 20.0, precision="bf16", tree=True, jitter=4)
    g.set_tree(None, None)
    with pytest.raises(F.FepllError, match="EINVAL"):
        F.select(g, x, 0.01, precision="bf16", tree=True)
