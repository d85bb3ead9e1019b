"""Pins of the jittered-subsampling reference (oracle/jitter.py, Sec. 3.3)."""
import os

import numpy as np
import pytest

import fepll_synth as fs
from oracle import epll64 as o
from oracle import jitter as j

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def test_philox_known_answers():
    rows = [l.split() for l in open(GOLDEN) if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(x, 16) for x in r]
        got = j.philox4x32_10(np.array(v[:4], np.uint64), v[4:6])
        assert [int(x) for x in got] == v[6:10]


def test_philox_is_a_bijection_of_the_counter():
    # distinct counters under one key give distinct outputs (it is a
    # keyed permutation of 128-bit blocks); a spot check over 2^16 counters
    ctr = np.zeros((1 << 16, 4), np.uint64)
    ctr[:, 0] = np.arange(1 << 16)
    out = j.philox4x32_10(ctr, (12345, 678))
    packed = {tuple(r) for r in out.tolist()}
    assert len(packed) == 1 << 16


@pytest.mark.parametrize("s", range(1, 9))
def test_grid_axis_spans_the_patch_range(s):
    b = (8 - s) // 2
    for n in (1, 2, 7, 33, 100):
        for g in range(s):
            a = j.grid_axis(n, s, g)
            assert a[0] <= -b < a[0] + s            # first point clamps to 0
            assert a[-1] - b >= n - 1                # last clamps to n - 1
            assert a.size == 1 or a[-2] - b < n - 1  # and no point beyond
            assert np.all(np.diff(a) == s)
            assert np.all((a - g) % s == 0)


@pytest.mark.parametrize("s", [2, 3, 4, 5, 6, 7, 8])
def test_every_pixel_covered_and_jitter_bounded(s):
    rng = np.random.default_rng(s)
    b = (8 - s) // 2
    for trial in range(20):
        H, W = int(rng.integers(8, 70)), int(rng.integers(8, 70))
        seed, t = int(rng.integers(0, 2 ** 63)), int(rng.integers(0, 16))
        idx, gr = j.positions(H, W, s, seed, t)
        Hp, Wp = H - 7, W - 7
        assert np.all(np.diff(idx) > 0) and idx[0] >= 0 and idx[-1] < Hp * Wp
        cov = np.zeros((H, W), int)
        for i in idx:
            r, c = divmod(int(i), Wp)
            cov[r:r + 8, c:c + 8] += 1
        assert cov.min() >= 1, (H, W, s, seed, t)
        # each point's start lies within b of its grid point, or is clamped
        R = gr["rows"][:, None] + np.zeros_like(gr["r"])
        C = gr["cols"][None, :] + np.zeros_like(gr["c"])
        okr = (np.abs(gr["r"] - R) <= b) | (gr["r"] == 0) | (gr["r"] == Hp - 1)
        okc = (np.abs(gr["c"] - C) <= b) | (gr["c"] == 0) | (gr["c"] == Wp - 1)
        assert okr.all() and okc.all()


def test_offsets_and_shift_are_uniform():
    """Over many iterations the shift takes every value in {0..s-1} and the
    interior offsets every value in {-b..b}, with frequencies within a few
    standard deviations of uniform."""
    s, b = 4, 2
    shifts = np.zeros(s, int)
    offs = np.zeros(2 * b + 1, int)
    for t in range(400):
        _, gr = j.positions(200, 200, s, 99, t)
        shifts[gr["gy"]] += 1
        rows = gr["rows"][:, None] + np.zeros_like(gr["r"])
        inner = (rows - b > 0) & (rows + b < 193)
        d = (gr["r"] - rows)[inner]
        offs += np.bincount(d + b, minlength=2 * b + 1)
    assert shifts.min() > 0
    p = offs / offs.sum()
    sd = np.sqrt(p * (1 - p) / offs.sum())
    assert np.all(np.abs(p - 1 / (2 * b + 1)) < 5 * sd + 1e-3), p


def test_subset_size_near_one_in_s_squared():
    H = W = 515
    for s in (3, 6):
        n = np.mean([j.positions(H, W, s, 7, t)[0].size for t in range(5)])
        assert 0.8 * (H - 7) * (W - 7) / s ** 2 < n < 1.3 * (H - 7) * (W - 7) / s ** 2


def test_all_patches_subset_is_plain_alg1():
    """With every patch in the subset, the subset iteration is Alg. 1."""
    c = fs.config_c1()
    x = c["y"][:30, :26]
    beta = 4.0 / c["sigma"] ** 2
    Hp, Wp = 23, 19
    want, wi = o.hqs_iteration(x, x, c["U"], c["lam"], c["w"], c["sigma"], beta)
    got, gi = j.hqs_iteration(x, x, c["U"], c["lam"], c["w"], c["sigma"], beta,
                              np.arange(Hp * Wp))
    np.testing.assert_array_equal(gi["labels"], wi["labels"])
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-10)


def test_subset_reprojection_brute_force():
    """The subset average, pixel by pixel from its definition, on a tiny
    image with a hand-picked subset."""
    c = fs.config_c1()
    x = c["y"][:12, :13]
    beta = 2.0 / c["sigma"] ** 2
    Wp = 6
    idx = np.array([0, 3, 5, 4 * Wp + 0, 4 * Wp + 5, 2 * Wp + 2])
    got, info = j.hqs_iteration(x, x, c["U"], c["lam"], c["w"], c["sigma"], beta, idx)
    _, nu, gamma, L = o.eigen_terms(c["lam"], c["w"], beta)
    b = beta * c["sigma"] ** 2
    for (py, px) in [(0, 0), (5, 7), (11, 12), (6, 2), (3, 9)]:
        acc, n = 0.0, 0
        for i in idx:
            r, cc = divmod(int(i), Wp)
            if r <= py < r + 8 and cc <= px < cc + 8:
                z = x[r:r + 8, cc:cc + 8].ravel()
                m = z.mean()
                costs = [-2 * np.log(c["w"][k]) + np.sum(np.log(nu[k]))
                         + np.sum((c["U"][k].T @ (z - m)) ** 2 / nu[k]) for k in range(len(c["w"]))]
                k = int(np.argmin(costs))
                zh = c["U"][k] @ (gamma[k] * (c["U"][k].T @ (z - m))) + m
                acc += zh[8 * (py - r) + (px - cc)]
                n += 1
        assert n == info["count"][py, px]
        want = (x[py, px] + b * acc / n) / (1 + b)
        assert abs(got[py, px] - want) < 1e-9
