"""Failure handling and state of the restoration runtime on the GPU:

* out of device memory (a simulated cap on what the library may hold): the
  call reports ENOMEM, writes nothing, the handle keeps working, and
  destroying it returns every byte;
* resuming: five HQS iterations in one call equal, bit for bit, the first
  two in one call and the last three in another started from their result
  (float32, and bfloat16 with the learned proposal).
"""
import os

import numpy as np
import pytest

import fepll_synth as fs
from oracle import epll64 as o

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

ENOMEM = -2


@pytest.fixture(scope="module")
def F():
    import paper_1710_08124_amd as F
    F.lib()
    return F


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def test_out_of_memory_reported_and_nothing_leaks(F):
    c = fs.config_c1()
    y = dev(c["y"])
    base = F.memory_in_use()
    want = F.restore(F.GMM(c["U"], c["lam"], c["w"]), y, c["sigma"]).cpu().numpy()
    torch.cuda.synchronize()
    assert F.memory_in_use() == base  # (the handle above is gone)
    g = F.GMM(c["U"], c["lam"], c["w"])
    held = F.memory_in_use()
    assert held > base
    out = dev(np.full(c["y"].shape, -7.0))
    for extra in (0, 4096, 1 << 20):
        F.set_memory_limit(held + extra)
        try:
            with pytest.raises(F.FepllError) as e:
                F.restore(g, y, c["sigma"], out=out)
            assert e.value.status == ENOMEM
        finally:
            F.set_memory_limit(0)
        torch.cuda.synchronize()
        assert np.all(out.cpu().numpy() == -7.0)  # nothing written
    got = F.restore(g, y, c["sigma"]).cpu().numpy()
    np.testing.assert_array_equal(got, want)
    g.close()
    assert F.memory_in_use() == base


@pytest.mark.parametrize("path", ["fp32", "bf16+proposal"])
def test_resume_is_bitwise(F, path):
    c = fs.config_c2(25.0)
    y = dev(c["y"][100:260, 40:230])
    g = F.GMM(c["U"], c["lam"], c["w"])
    kw = {}
    if path != "fp32":
        blob = os.path.join(os.path.dirname(F.__file__), "data", "proposal_k200_gmm12.bin")
        g.load_proposal(open(blob, "rb").read())
        kw = dict(precision="bf16", proposal=True, top_m=8, margin=0.5)
    betas = o.default_betas(25.0)
    whole = F.restore(g, y, 25.0, **kw).cpu().numpy()
    x2 = F.restore(g, y, 25.0, betas=betas[:2], **kw)
    x5 = F.restore(g, y, 25.0, betas=betas[2:], init=x2, **kw).cpu().numpy()
    np.testing.assert_array_equal(x5, whole)
    g.close()
