"""Jittered stochastic patch subsampling (Sec. 3.3) on the GPU against the
FP64 reference (oracle/jitter.py).

* the patches chosen at every iteration equal the reference's, bit for bit
  (both sides draw them from Philox4x32-10 with the same key and counters);
* float32, teacher-forced on the subset: labels bit-exact (certified),
  one iteration's image within 1e-4; end to end: label mismatches only at
  the reference's near-ties, dPSNR < 0.01 dB; at full size (1024^2, K = 200)
  too, the subset being about 1/36 of the patches;
* bf16 / e4m3 list selections against their definitions (oracle/lowp.py)
  on the subset: labels equal except at the definition's near-ties;
* quality of every precision within 0.05 dB of the FP64 jittered
  reference; a batch equals its images restored one by one."""
import math

import numpy as np
import pytest

import fepll_synth as fs
from oracle import epll64 as o
from oracle import jitter as jt
from oracle import lowp

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


@pytest.mark.parametrize("s", [1, 3, 6, 8])
@pytest.mark.parametrize("shape", [(64, 64), (71, 133), (8, 8), (40, 9)])
def test_positions_match_reference(F, s, shape):
    H, W = shape
    U, lam, w = fs.gmm(5, 3)
    g = F.GMM(U, lam, w)
    y = fs.noisy(fs.test_image(H, W, 7) if min(H, W) >= 16 else fs.dead_leaves(H, W, 7), 20.0, 8)
    seed = 0x1234_5678_9ABC_DEF0 + s
    _, lab = F.restore(g, dev(y), 20.0, precision="bf16", jitter=s, seed=seed,
                       return_labels=True)
    lab = lab.cpu().numpy()
    for t in range(5):
        want, _ = jt.positions(H, W, s, seed, t)
        got = np.nonzero(lab[t] < 5)[0]
        np.testing.assert_array_equal(got, want)


def _tf_fp32(F, y, U, lam, w, sigma, s, seed0):
    g = F.GMM(U, lam, w)
    y32 = f32(y)
    x = y32.copy()
    yd = dev(y32)
    H, W = y.shape
    worst = 0.0
    for t, beta in enumerate(o.default_betas(sigma)):
        seed = seed0 + t  # one iteration per call: counter t = 0, a new seed each step
        idx, _ = jt.positions(H, W, s, seed, 0)
        want, info = jt.hqs_iteration(x, y32, U, lam, w, sigma, float(beta), idx)
        got, lab = F.restore(g, yd, sigma, betas=[beta], init=dev(x), jitter=s, seed=seed,
                             return_labels=True)
        lab = lab.cpu().numpy()[0]
        np.testing.assert_array_equal(np.nonzero(lab < U.shape[0])[0], idx)
        np.testing.assert_array_equal(lab[idx], info["labels"])
        err = np.abs(got.cpu().numpy().astype(np.float64) - want).max()
        worst = max(worst, err)
        assert err <= TOL, (t, err)
        x = f32(want)
    return worst


def test_fp32_teacher_forced_c1(F):
    c = fs.config_c1()
    for s in (3, 6):
        w = _tf_fp32(F, c["y"], c["U"], c["lam"], c["w"], c["sigma"], s, 100 + s)
        print(f"C1 s={s}: worst |gpu - oracle| {w:.3g}")


@pytest.mark.parametrize("sigma", [10.0, 50.0])
def test_fp32_teacher_forced_k200_crop(F, sigma):
    c = fs.config_c2(sigma, size=512)
    w = _tf_fp32(F, c["y"][100:230, 50:211], c["U"], c["lam"], c["w"], sigma, 6, 7)
    print(f"K=200 crop sigma {sigma} s=6: worst |gpu - oracle| {w:.3g}")


def _end_to_end(F, g, y, x, U, lam, w, sigma, s, seed, precision="fp32"):
    y32 = f32(y)
    ref, hist = jt.restore(y32, U, lam, w, sigma, s, seed, trace=True)
    got, lab = F.restore(g, dev(y32), sigma, precision=precision, jitter=s, seed=seed,
                         return_labels=True)
    got = got.cpu().numpy().astype(np.float64)
    lab = lab.cpu().numpy()
    agree = []
    for t in range(5):
        idx = hist[t]["idx"]
        np.testing.assert_array_equal(np.nonzero(lab[t] < U.shape[0])[0], idx)
        agree.append(float(np.mean(lab[t][idx] == hist[t]["labels"])))
        if precision == "fp32":
            bad = np.nonzero(lab[t][idx] != hist[t]["labels"])[0]
            gap = hist[t]["second"][bad] - hist[t]["best"][bad]
            assert np.all(gap < 1e-2), gap
    d = o.psnr(x, ref) - o.psnr(x, got)
    return ref, got, agree, d


def test_fp32_end_to_end_k200(F):
    c = fs.config_c2(25.0, size=512)
    y, x = c["y"][:200, :256], c["x"][:200, :256]
    g = F.GMM(c["U"], c["lam"], c["w"])
    ref, got, agree, d = _end_to_end(F, g, y, x, c["U"], c["lam"], c["w"], 25.0, 6, 11)
    print("s=6 end to end: agreement", np.round(agree, 5), "dPSNR", d,
          "max|diff|", np.abs(got - ref).max())
    assert min(agree) >= 0.995
    assert abs(d) < 0.01


def test_fp32_full_size_end_to_end(F):
    """1024^2, K = 200, sigma 25, s = 6: the whole restoration against the
    FP64 jittered reference (about 29 000 patches per iteration)."""
    c = fs.config_c3(1024)
    g = F.GMM(c["U"], c["lam"], c["w"])
    ref, got, agree, d = _end_to_end(F, g, c["y"], c["x"], c["U"], c["lam"], c["w"], 25.0, 6,
                                     2024)
    print("1024^2 s=6: agreement", np.round(agree, 5), "dPSNR", d)
    assert min(agree) >= 0.995
    assert abs(d) < 0.01


@pytest.mark.parametrize("mode,rho", [("fp8", None), ("fp8", 0.95), ("bf16", None)])
def test_list_full_size_sampled(F, mode, rho):
    """The benchmarked configurations: 1024^2, K = 200, sigma 25, s = 6
    (about 29 000 chosen patches; e4m3: one list workgroup per 128 entries,
    no component split), e4m3 plain and flat-tailed, bf16.  The chosen
    patches equal the reference's; the labels of 3000 sampled chosen patches
    agree with the mode's definition except at its near-ties."""
    from oracle import flat_tail as ft
    c = fs.config_c3()
    y32 = np.asarray(c["y"], np.float32)
    beta = float(o.default_betas(25.0)[0])
    g = F.GMM(c["U"], c["lam"], c["w"])
    lam, r = c["lam"], None
    if rho is not None:
        r = g.flat_tail(rho)
        lam, want_r = ft.flat_tail(c["lam"], rho)
        np.testing.assert_array_equal(r, want_r)
    seed = 20171023
    _, lab = F.restore(g, dev(y32), 25.0, betas=[beta], precision=mode, jitter=6, seed=seed,
                       return_labels=True)
    lab = lab.cpu().numpy()[0]
    idx, _ = jt.positions(1024, 1024, 6, seed, 0)
    np.testing.assert_array_equal(np.nonzero(lab < 200)[0], idx)
    sel = np.sort(fs.rng(3).choice(idx, 3000, replace=False))
    eps = {"bf16": 64 * 2.0 ** -24, "fp8": 2.0 ** -12}[mode]  # as in test_gpu_precision
    cost, bnd = lowp.lowp_costs(y32, c["U"], lam, c["w"], beta, mode, acc_eps=eps, rank=r,
                                patches=sel)
    srt = np.sort(cost, 1)
    gap = srt[:, 1] - srt[:, 0]
    tol = bnd.max(1)
    same = lab[sel] == cost.argmin(1)
    print(f"1024^2 {mode} list rho={rho}: {idx.size} chosen, sampled agreement {same.mean():.5f}")
    assert np.all(same | (gap <= 2 * tol))


@pytest.mark.parametrize("mode", ["bf16", "fp8"])
@pytest.mark.parametrize("s,shape", [(6, (96, 200)), (3, (40, 300)), (4, (71, 9))])
def test_lowp_list_selection_matches_definition(F, mode, s, shape):
    """One iteration from a float32 image: the list selection's labels on
    the subset against the mode's definition (differences only at the
    definition's near-ties)."""
    c = fs.config_c2(25.0)
    H, W = shape
    x = np.asarray(c["y"][150:150 + H, 90:90 + W], np.float32)
    beta = float(o.default_betas(25.0)[2])
    g = F.GMM(c["U"], c["lam"], c["w"])
    _, lab = F.restore(g, dev(x), 25.0, betas=[beta], precision=mode, jitter=s, seed=77,
                       return_labels=True)
    lab = lab.cpu().numpy()[0]
    idx, _ = jt.positions(H, W, s, 77, 0)
    np.testing.assert_array_equal(np.nonzero(lab < 200)[0], idx)
    eps = {"bf16": 64 * 2.0 ** -24, "fp8": 2.0 ** -12}[mode]  # as in test_gpu_precision
    cost, bnd = lowp.lowp_costs(x, c["U"], c["lam"], c["w"], beta, mode, acc_eps=eps)
    cost, bnd = cost[idx], bnd[idx]
    srt = np.sort(cost, 1)
    gap = srt[:, 1] - srt[:, 0]
    tol = bnd.max(1)
    same = lab[idx] == cost.argmin(1)
    print(f"{mode} s={s} {shape}: {idx.size} patches, agreement {same.mean():.5f}")
    assert np.all(same | (gap <= 2 * tol))


_REFS = {}


def _ref(sigma, s):
    key = (sigma, s)
    if key not in _REFS:
        c = fs.config_c2(sigma)
        x, y = c["x"][128:288, 192:352], f32(c["y"][128:288, 192:352])
        _REFS[key] = (c, x, y, jt.restore(y, c["U"], c["lam"], c["w"], sigma, s, 5),
                      o.restore(y, c["U"], c["lam"], c["w"], sigma))
    return _REFS[key]


@pytest.mark.parametrize("mode", ["fp32", "bf16", "fp8"])
@pytest.mark.parametrize("sigma", [10.0, 25.0, 50.0])
def test_quality_against_jittered_reference(F, mode, sigma):
    s = 6
    c, x, y32, ref_j, ref = _ref(sigma, s)
    g = F.GMM(c["U"], c["lam"], c["w"])
    got = F.restore(g, dev(y32), sigma, precision=mode, jitter=s, seed=5)
    got = got.cpu().numpy().astype(np.float64)
    d = o.psnr(x, ref_j) - o.psnr(x, got)
    print(f"{mode} sigma {sigma} s={s}: dPSNR vs FP64 jittered {d:+.4f} dB; jittered vs all "
          f"patches (FP64) {o.psnr(x, ref_j) - o.psnr(x, ref):+.4f} dB")
    assert abs(d) <= 0.05


@pytest.mark.parametrize("mode", ["fp32", "bf16", "fp8"])
def test_batch_equals_single_images(F, mode):
    U, lam, w = fs.gmm(200, 12)
    g = F.GMM(U, lam, w)
    shapes = [(40, 70), (64, 64), (33, 129), (8, 8), (100, 57)]
    sig = [15.0, 30.0, 45.0, 20.0, 8.0]
    ys = []
    for i, (H, W) in enumerate(shapes):
        x = fs.test_image(H, W, 900 + i) if min(H, W) >= 16 else fs.dead_leaves(H, W, 900 + i)
        ys.append(fs.noisy(x, sig[i], 950 + i))
    got = F.restore_batch(g, [dev(v) for v in ys], sig, precision=mode, jitter=6, seed=99)
    for i, v in enumerate(ys):
        one = F.restore(g, dev(v), sig[i], precision=mode, jitter=6, seed=99).cpu().numpy()
        np.testing.assert_array_equal(got[i].cpu().numpy(), one)


def test_graph_replay_equals_eager(F):
    c = fs.config_c1()
    g = F.GMM(c["U"], c["lam"], c["w"])
    y = dev(f32(c["y"]))
    eager = F.restore(g, y, c["sigma"], precision="fp8", jitter=6, seed=3, profile=True)
    eager = eager.cpu().numpy()
    for _ in range(3):
        r = F.restore(g, y, c["sigma"], precision="fp8", jitter=6, seed=3).cpu().numpy()
        np.testing.assert_array_equal(r, eager)
        torch.cuda.synchronize()


def test_flat_tail_with_jitter_runs_against_reference(F):
    """The two approximations together (Sec. 3.1 + 3.3) against the FP64
    jittered reference on the flat-tailed spectra."""
    from oracle import flat_tail as ft
    c = fs.config_c2(25.0)
    x, y32 = c["x"][128:288, 192:352], f32(c["y"][128:288, 192:352])
    lft, _ = ft.flat_tail(c["lam"], 0.95)
    ref = jt.restore(y32, c["U"], lft, c["w"], 25.0, 6, 5)
    g = F.GMM(c["U"], c["lam"], c["w"])
    g.flat_tail(0.95)
    for mode in ("fp32", "bf16", "fp8"):
        got = F.restore(g, dev(y32), 25.0, precision=mode, jitter=6, seed=5).cpu().numpy()
        d = o.psnr(x, ref) - o.psnr(x, got.astype(np.float64))
        print(f"flat tail + jitter {mode}: dPSNR {d:+.4f} dB")
        assert abs(d) <= 0.05


def test_bad_jitter_options(F):
    c = fs.config_c1()
    g = F.GMM(c["U"], c["lam"], c["w"])
    y = dev(f32(c["y"]))
    for s in (-1, 9):
        with pytest.raises(F.FepllError, match="EINVAL"):
            F.restore(g, y, c["sigma"], jitter=s)
    g.load_proposal(F.MLP(20, fs.mlp_init(20, 3)).serialize())
    with pytest.raises(F.FepllError, match="EUNSUPPORTED"):
        F.restore(g, y, c["sigma"], precision="bf16", proposal=True, jitter=6)
    assert math.isfinite(float(F.restore(g, y, c["sigma"], jitter=8).cpu().sum()))


@pytest.mark.parametrize("shape,mode", [((1024, 1024), "fp8"), ((4096, 1024), "bf16")])
def test_list_iteration_sampled_pixels(F, shape, mode):
    """One iteration of a reduced-precision list path at full size (K = 200,
    sigma 25, s = 6), through the sort, the patch estimation and the
    reprojection: at 600 sampled pixels the image equals the update of
    Alg. 1 with each covering chosen patch's estimate under the label the
    GPU chose -- the reduced-precision modes' binary16 estimate of
    oracle/lowp.py, within its float32 accumulation bound -- their average
    and the image update, within 1e-4 more.  The 1024^2 list (29 chunks of
    1024 entries) sorts with the tables inside its scatter; the 4096 x 1024
    one (116 chunks) with a launch of its own for the tables."""
    from oracle import lowp
    H, W = shape
    c = fs.config_c2(25.0)
    U, lam, w = c["U"], c["lam"], c["w"]
    x0 = fs.test_image(H, W, 41)
    y32 = f32(fs.noisy(x0, 25.0, 42))
    beta = float(o.default_betas(25.0)[1])
    seed = 4242
    g = F.GMM(U, lam, w)
    got, lab = F.restore(g, dev(y32), 25.0, betas=[beta], precision=mode, jitter=6, seed=seed,
                         return_labels=True)
    got = got.cpu().numpy().astype(np.float64)
    lab = lab.cpu().numpy()[0]
    idx, _ = jt.positions(H, W, 6, seed, 0)
    np.testing.assert_array_equal(np.nonzero(lab < 200)[0], idx)
    Wp = W - 7
    chosen = np.zeros((H - 7) * Wp, bool)
    chosen[idx] = True
    R = fs.rng(43)
    py, px = R.integers(0, H, 600), R.integers(0, W, 600)
    cover = []
    for yy, xx in zip(py, px):
        rr, cc = np.meshgrid(np.arange(max(yy - 7, 0), min(yy, H - 8) + 1),
                             np.arange(max(xx - 7, 0), min(xx, W - 8) + 1), indexing="ij")
        rr, cc = rr.ravel(), cc.ravel()
        on = chosen[rr * Wp + cc]
        assert np.any(on)  # every pixel covered
        cover.append((rr[on], cc[on]))
    need = np.unique(np.concatenate([r * Wp + c for r, c in cover]))
    est, bnd = lowp.lowp_estimates(y32.astype(np.float32), U, lam, w, beta, lab[need],
                                   acc_eps=64 * 2.0 ** -24, patches=need)
    row = {int(p): i for i, p in enumerate(need)}
    b = beta * 25.0 ** 2
    worst = 0.0
    for (yy, xx), (rr, cc) in zip(zip(py, px), cover):
        i = np.array([row[int(p)] for p in rr * Wp + cc])
        off = 8 * (yy - rr) + (xx - cc)
        xt = np.mean(est[i, off])
        tol = TOL + b / (1.0 + b) * np.mean(bnd[i, off])
        want = o.image_update(y32[yy, xx], xt, beta, 25.0)
        worst = max(worst, abs(got[yy, xx] - want) / tol)
    print(f"{mode} {H}x{W} list iteration: {idx.size} chosen, worst sampled pixel error / "
          f"tolerance {worst:.3f}")
    assert worst <= 1.0


def test_state_between_calls(F):
    """The subset flags and lists persist between calls (all flags zero
    after a complete restoration): a list-path restoration is unchanged by
    float32 and other list-path restorations run before it, on other
    images, with other seeds and iteration counts."""
    c = fs.config_c2(25.0)
    g = F.GMM(c["U"], c["lam"], c["w"])
    y = dev(c["y"][100:228, 60:250])
    other = dev(c["y"][300:397, 10:131])
    first = F.restore(g, y, 25.0, precision="fp8", jitter=6, seed=11).cpu().numpy()
    F.restore(g, other, 25.0, precision="fp32", jitter=4, seed=12)
    F.restore(g, other, 25.0, precision="bf16", jitter=3, seed=13,
              betas=list(o.default_betas(25.0)[:2]))
    F.restore(g, y, 25.0, precision="fp8", jitter=6, seed=14, betas=list(o.default_betas(25.0)[:3]))
    again = F.restore(g, y, 25.0, precision="fp8", jitter=6, seed=11).cpu().numpy()
    np.testing.assert_array_equal(again, first)


def test_headline_configuration_end_to_end(F):
    """e4m3 + flat tail (rho 0.95) + jitter s = 6, all 5 iterations, on a
    768^2 crop of the 1024^2 sigma 25 image: a list long enough (about
    16 600 patches, 135 workgroups) for the one-pass selection that also
    counts the labels for the list sort.  Every iteration's chosen patches
    equal the reference's; the result is within 0.05 dB of the FP64
    jittered restoration on the same flat-tailed spectra."""
    from oracle import flat_tail as ft
    c = fs.config_c3()
    x, y32 = c["x"][:768, :768], f32(c["y"][:768, :768])
    seed = 20171023
    lft, _ = ft.flat_tail(c["lam"], 0.95)
    ref = jt.restore(y32, c["U"], lft, c["w"], 25.0, 6, seed)
    g = F.GMM(c["U"], c["lam"], c["w"])
    g.flat_tail(0.95)
    got, lab = F.restore(g, dev(y32), 25.0, precision="fp8", jitter=6, seed=seed,
                         return_labels=True)
    lab = lab.cpu().numpy()
    for t in range(5):
        want, _ = jt.positions(768, 768, 6, seed, t)
        np.testing.assert_array_equal(np.nonzero(lab[t] < 200)[0], want)
    # the default execution (graph replay) gives the eager result
    again = F.restore(g, dev(y32), 25.0, precision="fp8", jitter=6, seed=seed)
    eager = F.restore(g, dev(y32), 25.0, precision="fp8", jitter=6, seed=seed, profile=True)
    np.testing.assert_array_equal(again.cpu().numpy(), eager.cpu().numpy())
    np.testing.assert_array_equal(got.cpu().numpy(), eager.cpu().numpy())
    d = o.psnr(x, ref) - o.psnr(x, eager.cpu().numpy().astype(np.float64))
    print(f"headline configuration 768^2: dPSNR vs FP64 jittered flat tail {d:+.4f} dB")
    assert abs(d) <= 0.05
