"""Deblurring (a periodic convolution A, Alg. 1's image estimation in the
Fourier basis, Sec. 5's schedule and start) on the GPU against the FP64
reference (oracle/deblur.py).

* float32, teacher-forced: labels bit-exact (certified), one iteration's
  image within 1e-4 (the float64 FFTs add nothing measurable);
* the default schedule (lambda) and start end to end: label mismatches only
  at the reference's near-ties, dPSNR < 0.01 dB;
* the identity kernel is denoising; reduced precisions within 0.05 dB of
  the FP64 reference; invalid operators rejected."""
import ctypes

import numpy as np
import pytest

import fepll_synth as fs
from oracle import deblur as db
from oracle import epll64 as o

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-4


@pytest.fixture(scope="module")
def F():
    import paper_1710_08124_amd as F
    F.lib()
    return F


@pytest.fixture(scope="module")
def prob():
    return fs.config_deblur(size=96)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def f32(a):
    return np.asarray(a, np.float32).astype(np.float64)


def test_teacher_forced_fp32(F, prob):
    c = prob
    y32 = f32(c["y"])
    H, W = y32.shape
    g = F.GMM(c["U"], c["lam"], c["w"])
    x = f32(db.initial_estimate(y32, c["h"], c["sigma"]))
    worst = 0.0
    for t, beta in enumerate(db.default_betas(c["h"], H, W, c["sigma"])):
        want, info = db.hqs_iteration(x, y32, c["h"], c["U"], c["lam"], c["w"], c["sigma"],
                                      float(beta))
        got, lab = F.restore(g, dev(y32), c["sigma"], betas=[beta], init=dev(x), blur=c["h"],
                             return_labels=True)
        lab = lab.cpu().numpy()[0]
        mism = np.nonzero(lab != info["labels"])[0]
        assert mism.size == 0, (t, mism[:10])
        err = np.abs(got.cpu().numpy().astype(np.float64) - want).max()
        worst = max(worst, err)
        assert err <= TOL, (t, err)
        x = f32(want)
    print("deblur 96x96 K=200 teacher-forced: worst |gpu - oracle|", worst)


def test_default_schedule_and_start_end_to_end(F, prob):
    c = prob
    y32 = f32(c["y"])
    ref, hist = db.restore(y32, c["h"], c["U"], c["lam"], c["w"], c["sigma"], trace=True)
    g = F.GMM(c["U"], c["lam"], c["w"])
    got, lab = F.restore(g, dev(y32), c["sigma"], blur=c["h"], return_labels=True)
    got = got.cpu().numpy().astype(np.float64)
    lab = lab.cpu().numpy()
    agree = [float(np.mean(lab[t] == hist[t]["labels"])) for t in range(5)]
    for t in range(5):
        bad = np.nonzero(lab[t] != hist[t]["labels"])[0]
        gap = hist[t]["second"][bad] - hist[t]["best"][bad]
        assert np.all(gap < 1e-2), gap
    d = o.psnr(c["x"], ref) - o.psnr(c["x"], got)
    print("deblur end to end: agreement", np.round(agree, 5), "dPSNR", d,
          "PSNR y / restored", o.psnr(c["x"], y32), o.psnr(c["x"], ref))
    assert min(agree) >= 0.995
    assert abs(d) < 0.01
    if min(agree) == 1.0:
        assert np.abs(got - ref).max() <= TOL


def test_identity_kernel_is_denoising(F):
    c = fs.config_c1()
    y = dev(f32(c["y"]))
    g = F.GMM(c["U"], c["lam"], c["w"])
    want = F.restore(g, y, c["sigma"]).cpu().numpy()
    got = F.restore(g, y, c["sigma"], blur=np.ones((1, 1)), betas=o.default_betas(c["sigma"]),
                    init=y).cpu().numpy()
    assert np.abs(got - want).max() <= TOL


@pytest.mark.parametrize("mode", ["bf16", "fp8"])
def test_reduced_precision_quality(F, mode):
    c = fs.config_deblur(size=160)
    y32 = f32(c["y"])
    ref = db.restore(y32, c["h"], c["U"], c["lam"], c["w"], c["sigma"])
    g = F.GMM(c["U"], c["lam"], c["w"])
    got = F.restore(g, dev(y32), c["sigma"], blur=c["h"], precision=mode)
    d = o.psnr(c["x"], ref) - o.psnr(c["x"], got.cpu().numpy().astype(np.float64))
    print(f"deblur {mode}: dPSNR vs FP64 {d:+.4f} dB")
    assert abs(d) <= 0.05


@pytest.mark.parametrize("mode", ["fp32", "fp8"])
def test_deblur_with_flat_tail_and_jitter(F, mode):
    """Deblurring on the flat-tailed mixture (Sec. 3.1) with jittered patch
    subsets (Sec. 3.3) against the FP64 reference composed of the same
    steps: the Sec. 5 start and schedule, at iteration t the patch steps on
    the oracle's subset of t with the flat spectra, then the Fourier image
    estimation.  float32: end to end within 1e-3 dB (the labels agree where
    the trajectories do); e4m3: within 0.05 dB."""
    from oracle import flat_tail as ft
    from oracle import jitter as jt
    c = fs.config_deblur(size=128)
    g = F.GMM(c["U"], c["lam"], c["w"])
    g.flat_tail(0.95)
    y32 = f32(c["y"])
    H, W = y32.shape
    lam_f, _ = ft.flat_tail(c["lam"], 0.95)
    x = db.initial_estimate(y32, c["h"], c["sigma"])
    for t, beta in enumerate(db.default_betas(c["h"], H, W, c["sigma"])):
        idx, _ = jt.positions(H, W, 6, 1, t)
        xt, _ = jt.subset_estimate(x, c["U"], lam_f, c["w"], float(beta), idx)
        x = db.image_update(y32, xt, c["h"], float(beta), c["sigma"])
    got = F.restore(g, dev(y32), c["sigma"], blur=c["h"], precision=mode, jitter=6, seed=1)
    got = got.cpu().numpy().astype(np.float64)
    d = o.psnr(c["x"], x) - o.psnr(c["x"], got)
    print(f"deblur {mode} + flat + jitter: dPSNR vs FP64 {d:+.5f} dB "
          f"(blurred {o.psnr(c['x'], y32):.2f} dB, restored {o.psnr(c['x'], got):.2f} dB)")
    assert abs(d) <= (1e-3 if mode == "fp32" else 0.05)


def test_bad_operators_rejected(F, prob):
    c = prob
    g = F.GMM(c["U"], c["lam"], c["w"])
    y = dev(f32(c["y"]))
    with pytest.raises(F.FepllError, match="EINVAL"):
        F.restore(g, y, c["sigma"], blur=np.ones((4, 5)) / 20)  # even size
    with pytest.raises(F.FepllError, match="EINVAL"):
        F.restore(g, y, c["sigma"], blur=np.ones((97, 3)) / 291)  # taller than the image
    with pytest.raises(F.FepllError, match="EINVAL"):
        F.restore(g, y, c["sigma"], blur=np.full((3, 3), np.nan))
    yi = F._image(y)
    oi = F._image(torch.empty_like(y))
    op = F.Operator(7, 1, 1, None)
    st = F.lib().fepll_restore(g.handle, ctypes.byref(yi), ctypes.byref(op), 1.0, None, 0,
                               ctypes.byref(oi), None, None)
    assert st == -1
