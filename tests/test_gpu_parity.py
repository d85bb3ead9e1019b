"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Teacher forcing: the oracle runs its own trajectory; every oracle iterate is
rounded to float32, and both sides start the next iteration from that same
float32 image.  Labels must then be identical (the float32 selection
certifies each patch or re-selects it in float64), and one iteration's image
must agree to 1e-4 on the [0, 255] scale.
"""
import math

import numpy as np
import pytest

import fepll_synth as fs
from oracle import epll64 as o

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-4


@pytest.fixture(scope="module")
def F():
    import paper_1710_08124_amd as F
    F.lib()
    return F


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def f32(a):
    return np.asarray(a, np.float32).astype(np.float64)


def teacher_forced(F, y, U, lam, w, sigma, betas=None):
    """Run the oracle trajectory and compare one GPU iteration per step."""
    g = F.GMM(U, lam, w)
    betas = o.default_betas(sigma) if betas is None else np.asarray(betas)
    y32 = f32(y)
    x = y32.copy()
    yd = dev(y32)
    worst = 0.0
    for t, beta in enumerate(betas):
        want, info = o.hqs_iteration(x, y32, U, lam, w, sigma, float(beta))
        got, lab = F.restore(g, yd, sigma, betas=[beta], init=dev(x), return_labels=True)
        torch.cuda.synchronize()
        lab = lab.cpu().numpy()[0]
        mism = np.nonzero(lab != info["labels"])[0]
        assert mism.size == 0, (t, mism[:10], lab[mism[:10]], info["labels"][mism[:10]])
        err = np.abs(got.cpu().numpy().astype(np.float64) - want).max()
        worst = max(worst, err)
        assert err <= TOL, (t, err)
        x = f32(want)
    g.close()
    return worst


def test_teacher_forced_c1(F):
    c = fs.config_c1()
    print("C1 64x64 K=20 sigma=20")
    teacher_forced(F, c["y"], c["U"], c["lam"], c["w"], c["sigma"])


@pytest.mark.parametrize("H,W,K", [(71, 133, 7), (8, 8, 5), (8, 40, 3), (37, 8, 3),
                                   (15, 15, 1), (100, 71, 33)])
def test_teacher_forced_ragged_and_edges(F, H, W, K):
    print(f"ragged H={H} W={W} K={K}")
    U, lam, w = fs.gmm(K, 40 + K)
    x = fs.test_image(H, W, 500 + H)
    y = fs.noisy(x, 25.0, 600 + W)
    teacher_forced(F, y, U, lam, w, 25.0)


@pytest.mark.parametrize("sigma", [10.0, 25.0, 50.0])
def test_teacher_forced_k200_crop(F, sigma):
    """The K=200 mixture of the 512^2 workload on a 96x104 crop."""
    print(f"K=200 crop sigma={sigma}")
    c = fs.config_c2(sigma, size=512)
    y = c["y"][200:296, 300:404]
    teacher_forced(F, y, c["U"], c["lam"], c["w"], sigma)


def test_end_to_end_c1(F):
    """Five iterations without teacher forcing: labels can only differ where
    the oracle's own margin is within float32 drift, and the PSNR gap to the
    oracle is far below 0.05 dB."""
    c = fs.config_c1()
    y32 = f32(c["y"])
    ref, hist = o.restore(y32, c["U"], c["lam"], c["w"], c["sigma"], trace=True)
    g = F.GMM(c["U"], c["lam"], c["w"])
    got, lab = F.restore(g, dev(y32), c["sigma"], return_labels=True)
    got = got.cpu().numpy().astype(np.float64)
    lab = lab.cpu().numpy()
    agree = np.mean([np.mean(lab[t] == hist[t]["labels"]) for t in range(5)])
    print("end-to-end label agreement", agree, "max abs", np.abs(got - ref).max())
    assert agree >= 0.999
    for t in range(5):
        bad = np.nonzero(lab[t] != hist[t]["labels"])[0]
        gap = hist[t]["second"][bad] - hist[t]["best"][bad]
        assert np.all(gap < 1e-2), gap
    assert abs(o.psnr(c["x"], got) - o.psnr(c["x"], ref)) < 0.01
    if agree == 1.0:
        assert np.abs(got - ref).max() <= TOL


def test_select_matches_oracle_and_bounds(F):
    """One selection step: labels equal the exact argmin; the float32 best
    cost is within 1e-3 relative of the float64 one."""
    c = fs.config_c2(25.0)
    y32 = f32(c["y"][:80, :90])
    beta = 8.0 / 625.0
    g = F.GMM(c["U"], c["lam"], c["w"])
    lab, best, second, flags = F.select(g, dev(y32), beta)
    _, info = o.hqs_iteration(y32, y32, c["U"], c["lam"], c["w"], 25.0, beta)
    np.testing.assert_array_equal(lab.cpu().numpy(), info["labels"])
    b32 = best.cpu().numpy().astype(np.float64)
    fl = flags.cpu().numpy()
    ok = fl == 0
    np.testing.assert_allclose(b32[ok], info["best"][ok], rtol=1e-4)
    print("flagged fraction", fl.mean())


def test_no_recheck_differs_only_on_flagged(F):
    c = fs.config_c2(50.0)
    y32 = f32(c["y"][100:180, 40:140])
    beta = 1.0 / 2500.0
    g = F.GMM(c["U"], c["lam"], c["w"])
    lab0, _, _, fl = F.select(g, dev(y32), beta, recheck=False)
    lab1, _, _, _ = F.select(g, dev(y32), beta, recheck=True)
    diff = (lab0 != lab1).cpu().numpy()
    assert np.all(fl.cpu().numpy()[diff] == 1)


def test_deterministic_and_host_device_paths_agree(F):
    c = fs.config_c1()
    y32 = np.ascontiguousarray(c["y"], np.float32)
    g = F.GMM(c["U"], c["lam"], c["w"])
    a = F.restore(g, dev(y32), 20.0).cpu().numpy()
    b = F.restore(g, dev(y32), 20.0).cpu().numpy()
    h = F.restore(g, y32, 20.0)
    np.testing.assert_array_equal(a, b)
    np.testing.assert_array_equal(a, h)


def test_strided_and_aliased_images(F):
    c = fs.config_c1()
    big = torch.zeros((64, 80), dtype=torch.float32, device="cuda")
    big[:, 5:69] = dev(c["y"])
    view = big[:, 5:69]
    g = F.GMM(c["U"], c["lam"], c["w"])
    ref = F.restore(g, dev(c["y"]), 20.0)
    F.restore(g, view, 20.0, out=view)   # in place on a strided view
    np.testing.assert_array_equal(view.cpu().numpy(), ref.cpu().numpy())


def test_error_paths(F):
    c = fs.config_c1()
    g = F.GMM(c["U"], c["lam"], c["w"])
    y = dev(c["y"])
    import ctypes
    yi = F._image(y)
    oi = F._image(torch.empty_like(y))
    op = F.Operator(99, 1, 1, None)  # an operator kind the library does not know
    st = F.lib().fepll_restore(g.handle, ctypes.byref(yi), ctypes.byref(op), 20.0, None, 0,
                               ctypes.byref(oi), None, None)
    assert st == -1
    bad = np.array(c["y"], np.float32)
    bad[3, 4] = np.nan
    with pytest.raises(F.FepllError):
        F.restore(g, bad, 20.0)
    with pytest.raises(F.FepllError):
        F.restore(g, y, -1.0)
    with pytest.raises(F.FepllError):
        F.restore(g, y, 20.0, betas=[1.0, -2.0])
    with pytest.raises(F.FepllError):
        F.restore(g, dev(np.zeros((7, 20))), 20.0)


@pytest.mark.parametrize("seed", [0])
def test_full_size_first_iteration_sampled(F, seed):
    """1024^2, K=200, sigma=25, first iteration (x = y): the labels of 3000
    sampled patches and the restored value of 60 sampled pixels against the
    oracle computed patch by patch."""
    c = fs.config_c3()
    y32 = f32(c["y"])
    U, lam, w = c["U"], c["lam"], c["w"]
    sigma = 25.0
    beta = 1.0 / sigma ** 2
    g = F.GMM(U, lam, w)
    yd = dev(y32)
    got, lab = F.restore(g, yd, sigma, betas=[beta], return_labels=True)
    got = got.cpu().numpy().astype(np.float64)
    lab = lab.cpu().numpy()[0]
    H = W = 1024
    Wp = W - 7
    rng = fs.rng(seed)
    idx = rng.choice((H - 7) * Wp, 3000, replace=False)
    r, cc = idx // Wp, idx % Wp
    Z = o.extract(y32, r, cc)
    Zt, m = o.remove_dc(Z)
    _, nu, gamma, L = o.eigen_terms(lam, w, beta)
    want = np.argmin(o.selection_costs(Zt, U, nu, L), axis=1)
    np.testing.assert_array_equal(lab[idx], want)
    # pixels: every covering patch's estimate, averaged, then the update
    pix = rng.integers(0, H, (60, 2))
    for (py, px) in pix:
        rr, c2 = np.meshgrid(np.arange(max(0, py - 7), min(H - 8, py) + 1),
                             np.arange(max(0, px - 7), min(W - 8, px) + 1), indexing="ij")
        rr, c2 = rr.ravel(), c2.ravel()
        Z = o.extract(y32, rr, c2)
        Zt, m = o.remove_dc(Z)
        k = np.argmin(o.selection_costs(Zt, U, nu, L), axis=1)
        Zh = o.patch_estimate(Zt, m, k, U, gamma)
        vals = Zh[np.arange(rr.size), 8 * (py - rr) + (px - c2)]
        want_px = o.image_update(y32[py, px], vals.mean(), beta, sigma)
        assert abs(got[py, px] - want_px) <= TOL, (py, px, got[py, px], want_px)


def test_mixture_from_covariances(F):
    """fepll_gmm_create_from_cov (float64 Jacobi eigendecomposition in the
    library) restores like the mixture given by its eigendecomposition: the
    eigenvectors differ at most in sign, which the costs (squares) and the
    Wiener filters U diag(gamma) U^t do not see."""
    c = fs.config_c1()
    U, lam, w = c["U"], c["lam"], c["w"]
    Sigma = U @ (lam[:, :, None] * U.transpose(0, 2, 1))
    g0 = F.GMM(U, lam, w)
    g1 = F.GMM.from_cov(Sigma, w)
    y = dev(f32(c["y"]))
    a, la = F.restore(g0, y, c["sigma"], return_labels=True)
    b, lb = F.restore(g1, y, c["sigma"], return_labels=True)
    agree = float((la == lb).float().mean().item())
    err = float((a - b).abs().max().item())
    print("labels agree", agree, "max |diff|", err)
    assert agree >= 0.999 and err <= 1e-3
