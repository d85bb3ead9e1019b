"""Pins of the flat-tail reference (oracle/flat_tail.py, Sec. 3.1)."""
import numpy as np
import pytest

import fepll_synth as fs
from oracle import epll64 as o
from oracle import flat_tail as ft


def test_flat_tail_definition():
    _, lam, _ = fs.gmm(20, 11)
    for rho in (0.5, 0.9, 0.95, 0.99):
        lft, r = ft.flat_tail(lam, rho)
        for k in range(lam.shape[0]):
            rk = r[k]
            tot = lam[k].sum()
            assert lam[k, :rk].sum() >= rho * tot
            assert rk == 1 or lam[k, :rk - 1].sum() < rho * tot  # smallest such rank
            np.testing.assert_array_equal(lft[k, :rk], lam[k, :rk])
            np.testing.assert_allclose(lft[k].sum(), tot, rtol=1e-13)  # trace kept
            if rk < 64:
                assert np.all(lft[k, rk:] == lft[k, rk])  # flat tail
                assert np.all(np.diff(lft[k]) <= 1e-12 * tot)  # still decreasing
    lft, r = ft.flat_tail(lam, 1.0)
    np.testing.assert_array_equal(lft, lam)


def test_synthetic_ranks():
    """The K=200 mixture at rho = 0.95: the ranks the kernels rely on."""
    _, lam, _ = fs.gmm(200, 12)
    _, r = ft.flat_tail(lam, 0.95)
    print("ranks: mean", r.mean(), "max", r.max(), "min", r.min())
    assert 4 <= r.mean() <= 20 and r.max() <= 32


@pytest.mark.parametrize("rho", [0.8, 0.95, 1.0])
def test_rewritten_selection_equals_plain_cost(rho):
    """Sec. 3.1's selection form (r_k projections + |z~|^2) equals the plain
    eigenspace cost of epll64 on the flat-tailed spectrum."""
    c = fs.config_c1()
    x = c["y"][10:30, 5:29]
    r_, c_ = o.patch_corners(*x.shape)
    Zt, _ = o.remove_dc(o.extract(x, r_, c_))
    lft, r = ft.flat_tail(c["lam"], rho)
    for beta in (1 / 400.0, 32 / 400.0):
        _, nu, _, L = o.eigen_terms(lft, c["w"], beta)
        want = o.selection_costs(Zt, c["U"], nu, L)
        got = ft.flat_tail_costs(Zt, c["U"], lft, r, c["w"], beta)
        np.testing.assert_allclose(got, want, rtol=1e-11, atol=1e-9)


@pytest.mark.parametrize("rho", [0.8, 0.95])
def test_rewritten_estimate_equals_plain_estimate(rho):
    c = fs.config_c1()
    x = c["y"][:20, :20]
    r_, c_ = o.patch_corners(*x.shape)
    Zt, m = o.remove_dc(o.extract(x, r_, c_))
    lft, r = ft.flat_tail(c["lam"], rho)
    beta = 4 / 400.0
    _, nu, gam, L = o.eigen_terms(lft, c["w"], beta)
    lab = o.select(o.selection_costs(Zt, c["U"], nu, L))[0]
    want = o.patch_estimate(Zt, m, lab, c["U"], gam)
    got = ft.flat_tail_estimate(Zt, m, lab, c["U"], lft, r, beta)
    np.testing.assert_allclose(got, want, rtol=1e-11, atol=1e-9)


def test_flat_tail_limits():
    """rho = 1 is EPLL itself; a smaller rho changes the restoration by a
    bounded amount on the small workload."""
    c = fs.config_c1()
    y = c["y"][:24, :24]
    a = o.restore(y, c["U"], c["lam"], c["w"], c["sigma"])
    b = ft.restore(y, c["U"], c["lam"], c["w"], c["sigma"], 1.0)
    np.testing.assert_array_equal(a, b)
    d = ft.restore(y, c["U"], c["lam"], c["w"], c["sigma"], 0.95)
    assert 0 < np.abs(d - a).max() < 255
