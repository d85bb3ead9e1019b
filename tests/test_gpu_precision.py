"""Reduced-precision projections (bfloat16) against the FP64 oracle.

In this mode the selection is an approximation: the tests state its label
agreement with the exact selection and bound its PSNR loss, which is the
quality criterion of the mode (within 0.05 dB of the FP64 oracle)."""
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


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def f32(a):
    return np.asarray(a, np.float32).astype(np.float64)


@pytest.mark.parametrize("case", ["c1", "k200_10", "k200_25", "k200_50"])
def test_bf16_quality(F, case):
    if case == "c1":
        c = fs.config_c1()
        x, y = c["x"], c["y"]
    else:
        sigma = float(case.split("_")[1])
        c = fs.config_c2(sigma)
        x, y = c["x"][128:288, 192:352], c["y"][128:288, 192:352]
    sigma = c["sigma"]
    y32 = f32(y)
    ref, hist = o.restore(y32, c["U"], c["lam"], c["w"], sigma, trace=True)
    g = F.GMM(c["U"], c["lam"], c["w"])
    got, lab = F.restore(g, dev(y32), sigma, precision="bf16", return_labels=True)
    got = got.cpu().numpy().astype(np.float64)
    lab = lab.cpu().numpy()
    # teacher-forced first iteration: agreement of the selection alone
    agree0 = float(np.mean(lab[0] == hist[0]["labels"]))
    agree = [float(np.mean(lab[t] == hist[t]["labels"])) for t in range(5)]
    dpsnr = o.psnr(x, ref) - o.psnr(x, got)
    print(f"{case}: label agreement first iteration {agree0:.4f}, per iteration "
          f"{np.round(agree, 4).tolist()}, dPSNR {dpsnr:+.4f} dB, "
          f"max|diff| {np.abs(got - ref).max():.3f}")
    assert agree0 > 0.9
    assert abs(dpsnr) <= 0.05


def test_bf16_select_shape_and_range(F):
    c = fs.config_c1()
    g = F.GMM(c["U"], c["lam"], c["w"])
    lab, best, second, flags = F.select(g, dev(c["y"]), 1 / 400.0, precision="bf16")
    lab = lab.cpu().numpy()
    assert lab.min() >= 0 and lab.max() < 20
    assert np.all(second.cpu().numpy() >= best.cpu().numpy())
    assert not flags.cpu().numpy().any()
