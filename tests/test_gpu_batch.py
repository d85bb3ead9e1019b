"""Batched restoration (fepll_restore_batch), graph replay and the autotuner.

A batch packs images of uneven sizes, each with its own noise level (so its
own betas), and runs every stage of an iteration as one launch over all of
them.  Per patch the arithmetic is the one of a single-image restoration,
so every image of a batch must equal, bit for bit, the image restored on
its own; and the float32 batch must match the FP64 oracle like the
single-image path does.  Replays of the captured graph must equal the eager
run, with other GPU work between the replays, and so must every launch
shape the autotuner may pick."""
import numpy as np
import pytest

import fepll_synth as fs
from oracle import epll64 as o

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def F():
    import paper_1710_08124_amd as F
    F.lib()
    return F


@pytest.fixture(scope="module")
def gm():
    return fs.gmm(200, 12)


# uneven shapes, a single-patch image and a single patch column included
SHAPES = [(40, 70), (64, 64), (33, 129), (100, 57), (8, 8), (71, 8)]
SIGMAS = [15.0, 30.0, 45.0, 8.0, 20.0, 35.0]


@pytest.fixture(scope="module")
def small_batch():
    out = []
    for i, ((H, W), s) in enumerate(zip(SHAPES, SIGMAS)):
        x = fs.test_image(H, W, 900 + i) if min(H, W) >= 16 else fs.dead_leaves(H, W, 900 + i)
        out.append(dict(x=x, y=fs.noisy(x, s, 950 + i), sigma=s))
    return out


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def single(F, g, b, **kw):
    return [F.restore(g, dev(d["y"]), d["sigma"], **kw).cpu().numpy() for d in b]


@pytest.mark.parametrize("mode", ["fp32", "bf16", "fp8"])
def test_batch_equals_single_images(F, gm, small_batch, mode):
    g = F.GMM(*gm)
    ys = [dev(d["y"]) for d in small_batch]
    got = F.restore_batch(g, ys, [d["sigma"] for d in small_batch], precision=mode)
    want = single(F, g, small_batch, precision=mode)
    for i, (a, b) in enumerate(zip(got, want)):
        print(f"{mode} image {i} {SHAPES[i]}: max |batch - single| "
              f"{np.abs(a.cpu().numpy() - b).max():.3g}")
        np.testing.assert_array_equal(a.cpu().numpy(), b)


def test_batch_fp32_matches_oracle(F, gm, small_batch):
    """End to end against the FP64 oracle, with the criterion of the
    single-image path: labels differ only where the oracle's own margin is
    within float32 drift, the PSNR gap is far below 0.05 dB, and images with
    no label difference agree to 1e-4."""
    g = F.GMM(*gm)
    ys = [dev(d["y"]) for d in small_batch]
    got = F.restore_batch(g, ys, [d["sigma"] for d in small_batch], precision="fp32")
    for i, d in enumerate(small_batch):
        y32 = np.asarray(d["y"], np.float32).astype(np.float64)
        ref, hist = o.restore(y32, gm[0], gm[1], gm[2], d["sigma"], trace=True)
        one, lab = F.restore(g, ys[i], d["sigma"], return_labels=True)
        np.testing.assert_array_equal(got[i].cpu().numpy(), one.cpu().numpy())
        lab = lab.cpu().numpy()
        out = got[i].cpu().numpy().astype(np.float64)
        err = np.abs(out - ref).max()
        agree = np.mean([np.mean(lab[t] == hist[t]["labels"]) for t in range(5)])
        print(f"image {i} {SHAPES[i]} sigma {d['sigma']}: label agreement {agree:.5f}, "
              f"max |gpu - oracle| {err:.3g}")
        assert agree >= 0.995
        for t in range(5):
            bad = np.nonzero(lab[t] != hist[t]["labels"])[0]
            gap = hist[t]["second"][bad] - hist[t]["best"][bad]
            assert np.all(gap < 1e-2), gap
        assert abs(o.psnr(d["x"], out) - o.psnr(d["x"], ref)) < 0.01
        if agree == 1.0:
            assert err <= 1e-4


def test_batch_host_images(F, gm, small_batch):
    g = F.GMM(*gm)
    ys = [np.asarray(d["y"], np.float32) for d in small_batch[:3]]
    got = F.restore_batch(g, ys, [d["sigma"] for d in small_batch[:3]], precision="bf16")
    want = single(F, g, small_batch[:3], precision="bf16")
    for a, b in zip(got, want):
        np.testing.assert_array_equal(a, b)


@pytest.mark.parametrize("mode", ["bf16", "fp32"])
def test_graph_replays_equal_eager(F, gm, small_batch, mode):
    g = F.GMM(*gm)
    sig = [d["sigma"] for d in small_batch]
    ys = [dev(d["y"]) for d in small_batch]
    eager = [t.cpu().numpy() for t in F.restore_batch(g, ys, sig, precision=mode, profile=True)]
    F.profile(g)
    junk = torch.randn(1 << 20, device="cuda")
    for rep in range(4):
        got = F.restore_batch(g, ys, sig, precision=mode)  # captured once, then replayed
        # other work on the stream and a host synchronisation between replays
        junk = junk * 0.5 + 1.0
        torch.cuda.synchronize()
        for i, (a, b) in enumerate(zip(got, eager)):
            assert np.array_equal(a.cpu().numpy(), b), f"replay {rep} image {i}"
    # a different call in between changes the plan: the next call captures anew
    F.select(g, ys[0], 1e-3, precision=mode)
    got = F.restore_batch(g, ys, sig, precision=mode)
    for a, b in zip(got, eager):
        np.testing.assert_array_equal(a.cpu().numpy(), b)


def test_single_restore_graph_equals_eager(F, gm, small_batch):
    g = F.GMM(*gm)
    y = dev(small_batch[2]["y"])
    s = small_batch[2]["sigma"]
    eager = F.restore(g, y, s, precision="fp8", profile=True).cpu().numpy()
    F.profile(g)
    for _ in range(3):
        np.testing.assert_array_equal(F.restore(g, y, s, precision="fp8").cpu().numpy(), eager)


def test_profile_stage_mask(F, gm, small_batch):
    """options.profile as a stage mask: only the named stages are timed,
    each as often as with every stage timed (a chained stage after an
    untimed one opens its own interval); the results are unchanged."""
    g = F.GMM(*gm)
    y = dev(small_batch[2]["y"])
    s = small_batch[2]["sigma"]
    kw = dict(precision="fp8", jitter=6, seed=7)
    F.restore(g, y, s, profile=True, **kw)  # (the first call also builds the constants)
    F.profile(g)
    ref = F.restore(g, y, s, profile=True, **kw).cpu().numpy()
    allst = F.profile(g)
    for stages in (["select"], ["wiener"], ["select", "ola_update"], ["bucket", "wiener"]):
        got = F.restore(g, y, s, profile=stages, **kw).cpu().numpy()
        np.testing.assert_array_equal(got, ref)
        p = F.profile(g)
        for k, (ms, n) in p.items():
            if k in stages:
                assert n == allst[k][1] and n > 0 and ms > 0.0, (stages, k, p[k], allst[k])
            else:
                assert n == 0, (stages, k, p[k])
    for bad in (-1, 2 << 9):
        with pytest.raises(F.FepllError, match="EINVAL"):
            F.restore(g, y, s, profile=bad, **kw)


def test_autotune_and_shapes_keep_results(F, gm, small_batch):
    g = F.GMM(*gm)
    sig = [d["sigma"] for d in small_batch]
    ys = [dev(d["y"]) for d in small_batch]
    ref = [t.cpu().numpy() for t in F.restore_batch(g, ys, sig, precision="bf16")]
    best = F.autotune(g, ys, sig, precision="bf16")
    print("tuned:", best)
    assert best["est_blocks"] in (0, 512, 768, 1024)
    assert best["wiener_blocks"] in (1024, 2048, 4096, 8192)
    assert best["ola_rows"] in (16, 32, 64)
    assert F.get_tuning(g) == best
    for shape in [dict(est_blocks=0, wiener_blocks=8, ola_rows=16),
                  dict(est_blocks=1, wiener_blocks=1024, ola_rows=64), best]:
        F.set_tuning(g, **shape)
        got = F.restore_batch(g, ys, sig, precision="bf16")
        for a, b in zip(got, ref):
            np.testing.assert_array_equal(a.cpu().numpy(), b)


def test_autotune_cache(F, gm, small_batch, tmp_path, monkeypatch):
    """FEPLL_TUNING_CACHE: a tuned workload is written once; the same kind of
    workload is then tuned from the file with no trial (no new line), the
    last line for a key winning; another precision is its own key."""
    path = tmp_path / "tuning.txt"
    monkeypatch.setenv("FEPLL_TUNING_CACHE", str(path))
    g = F.GMM(*gm)
    sig = [d["sigma"] for d in small_batch]
    ys = [dev(d["y"]) for d in small_batch]
    best = F.autotune(g, ys, sig, precision="bf16")
    lines = path.read_text().splitlines()
    assert len(lines) == 1 and lines[0].startswith("fepll-tuning 1 ")
    key = lines[0].split()[2]
    assert ":K200:" in key
    F.set_tuning(g, est_blocks=1, wiener_blocks=1024, ola_rows=16)
    assert F.autotune(g, ys, sig, precision="bf16") == best
    assert len(path.read_text().splitlines()) == 1
    with open(path, "a") as f:
        f.write(f"fepll-tuning 1 {key} 512 2048 64\n")
    assert F.autotune(g, ys, sig, precision="bf16") == dict(est_blocks=512, wiener_blocks=2048,
                                                            ola_rows=64)
    F.autotune(g, ys, sig, precision="fp8")
    lines = path.read_text().splitlines()
    assert len(lines) == 3 and lines[2].split()[2] != key
    g.close()


def test_batch_with_proposal_equals_single(F, gm, small_batch):
    import os
    path = os.path.join(os.path.dirname(F.__file__), "data", "proposal_k200_gmm12.bin")
    g = F.GMM(*gm)
    g.load_proposal(open(path, "rb").read())
    kw = dict(precision="bf16", proposal=True, top_m=8, margin=0.5)
    ys = [dev(d["y"]) for d in small_batch]
    got = F.restore_batch(g, ys, [d["sigma"] for d in small_batch], **kw)
    want = single(F, g, small_batch, **kw)
    for a, b in zip(got, want):
        np.testing.assert_array_equal(a.cpu().numpy(), b)


def test_large_uneven_batch_sampled(F, gm):
    """Image sizes of the 48-image workload (256^2 up to 1024 x 1536, so the
    octile-major tile tables of several images in one launch): the batch
    against single-image restorations of the same images, bit for bit, in
    every precision and with the learned proposal (its fallback search
    split over halves of K across images)."""
    import os
    g = F.GMM(*gm)
    g.load_proposal(open(os.path.join(os.path.dirname(F.__file__), "data",
                                      "proposal_k200_gmm12.bin"), "rb").read())
    shapes = [(256, 256), (1024, 1536), (517, 901), (300, 1200)]
    sig = [7.5, 42.0, 25.0, 13.0]
    b = []
    for i, (H, W) in enumerate(shapes):
        x = fs.test_image(H, W, 700 + i)
        b.append(dict(y=fs.noisy(x, sig[i], 800 + i), sigma=sig[i]))
    ys = [dev(d["y"]) for d in b]
    for kw in (dict(precision="bf16"), dict(precision="fp8"), dict(precision="fp32"),
               dict(precision="bf16", proposal=True, top_m=8, margin=0.5)):
        got = F.restore_batch(g, ys, sig, **kw)
        want = single(F, g, b, **kw)
        for a, w in zip(got, want):
            np.testing.assert_array_equal(a.cpu().numpy(), w)


def test_batch_rejects_bad_arguments(F, gm, small_batch):
    g = F.GMM(*gm)
    ys = [dev(d["y"]) for d in small_batch[:2]]
    with pytest.raises(F.FepllError, match="EINVAL"):
        F.restore_batch(g, ys, [10.0, -1.0])
    with pytest.raises(F.FepllError, match="EINVAL"):
        F.restore_batch(g, ys, [10.0, 20.0], outs=[torch.empty(5, 5, device="cuda")] * 2)
    with pytest.raises(F.FepllError, match="EINVAL"):
        F.set_tuning(g, wiener_blocks=12)
    with pytest.raises(F.FepllError, match="EINVAL"):
        F.set_tuning(g, ola_rows=24)
    with pytest.raises(F.FepllError, match="EINVAL|EUNSUPPORTED"):
        F.restore_batch(g, ys, [10.0, 20.0], precision="fp8", proposal=True)
