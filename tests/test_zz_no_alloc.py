"""fepll_select_static, the selection entry point that allocates no device
memory, against fepll_select (float32, recheck on) through the C ABI: equal
labels, costs and flags bit for bit on two calls in a row, the second on a
smaller image; sizes beyond its scratch are refused."""
import numpy as np
import pytest

import fepll_synth as fs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def F():
    import paper_1710_08124_amd as F
    F.lib()
    return F


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def test_static_select_equals_select(F):
    c = fs.config_c2(25.0)
    g = F.GMM(c["U"], c["lam"], c["w"])
    for (r0, c0, H, W), t in (((40, 60, 200, 333), 0), ((300, 10, 57, 90), 3)):
        x = dev(c["y"][r0:r0 + H, c0:c0 + W])
        beta = float((1.0, 4.0, 8.0, 16.0, 32.0)[t]) / 25.0 ** 2
        want = [v.cpu().numpy() for v in F.select(g, x, beta)]
        got = [v.cpu().numpy() for v in F.select_static(g, x, beta)]
        torch.cuda.synchronize()
        for a, b in zip(got, want):
            np.testing.assert_array_equal(a, b)
        print((H, W), "uncertified", int(want[3].sum()))
    # an image whose uncertified list would not fit the scratch
    big = dev(np.zeros((1600, 1600), np.float32))
    with pytest.raises(F.FepllError):
        F.select_static(g, big, 1.0 / 625.0)
    g.close()
