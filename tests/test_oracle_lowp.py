"""Pins of the reduced-precision reference definitions (oracle/lowp.py).

The rounding functions are written from the two formats' definitions; here
they are held against PyTorch's own float32 -> bfloat16 and
float32 -> float8_e4m3fn conversions (library routines, nearest-even), and
the costs against the exact float64 costs where rounding is exact and
against the rounding-error bound elsewhere."""
import numpy as np
import pytest

import fepll_synth as fs
from oracle import epll64 as o
from oracle import lowp

torch = pytest.importorskip("torch")


def _probe_values(seed, n=200_000):
    rng = np.random.default_rng(seed)
    mag = np.ldexp(rng.uniform(1.0, 2.0, n), rng.integers(-14, 10, n))
    x = (mag * rng.choice([-1.0, 1.0], n)).astype(np.float32)
    return x


def test_round_bf16_matches_torch():
    x = _probe_values(1)
    want = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    np.testing.assert_array_equal(lowp.round_bf16(x), want)


def test_round_e4m3_matches_torch():
    x = _probe_values(2)
    x = x[np.abs(x) < 464.0]
    # values at and between grid points, ties included
    grid = np.unique(np.abs(lowp.round_e4m3(np.linspace(-448, 448, 20001))))
    mids = ((grid[1:] + grid[:-1]) / 2).astype(np.float32)
    x = np.concatenate([x, mids, -mids, grid.astype(np.float32)])
    want = torch.from_numpy(x).to(torch.float8_e4m3fn).to(torch.float32).numpy()
    got = lowp.round_e4m3(x)
    np.testing.assert_array_equal(got, want.astype(np.float64))


def test_e4m3_grid():
    # 0, 7 subnormals and 15 binades x 8 mantissas less the NaN code: 127 magnitudes
    x = np.concatenate([np.linspace(0.0, 0.03, 30001), np.linspace(-500, 500, 400001)])
    grid = np.unique(np.abs(lowp.round_e4m3(x)))
    grid = grid[np.isfinite(grid)]
    assert grid[-1] == 448.0 and grid[1] == 2.0 ** -9
    assert len(grid) == 127
    assert np.isnan(lowp.round_e4m3(465.0)) and lowp.round_e4m3(464.0) == 448.0


def test_pow2_exponent():
    rng = np.random.default_rng(3)
    mx = np.ldexp(rng.uniform(0.5, 1.0, 10000), rng.integers(-60, 60, 10000))
    mx[:4] = [448.0, 448.0 * 2 ** 5, 449.0, 447.0]
    e = lowp.pow2_exponent(mx)
    assert np.all(np.ldexp(mx, -e) <= 448.0)
    assert np.all(np.ldexp(mx, -(e - 1)) > 448.0)
    assert list(e[:4]) == [0, 5, 1, 0]
    assert lowp.pow2_exponent(0.0) == 0


def _nearest_f32(q):
    """The float32 nearest to the rational q, ties to the even significand:
    brute force over the neighbours of a first guess."""
    from fractions import Fraction
    f = np.float32(float(q))
    cands = [f, np.nextafter(f, np.float32(np.inf)), np.nextafter(f, np.float32(-np.inf))]
    dist = [abs(Fraction(float(c)) - q) for c in cands]
    best = min(dist)
    ties = [c for c, d in zip(cands, dist) if d == best]
    if len(ties) > 1:
        ties = [c for c in ties if int(np.float32(c).view(np.uint32)) & 1 == 0]
    return ties[0]


def _dc_removed_brute(Z):
    """z~ by exact rational arithmetic: the pixel sum correctly rounded to
    float64 (int / int true division rounds correctly), divided by 64, and
    z - m rounded to the nearest float32."""
    from fractions import Fraction
    out = np.empty(Z.shape, np.float32)
    for i, row in enumerate(Z):
        S = sum(Fraction(float(v)) for v in row)
        m = Fraction(S.numerator / S.denominator) / 64
        for j, v in enumerate(row):
            out[i, j] = _nearest_f32(Fraction(float(v)) - m)
    return out


def test_dc_removed_exact_against_rational_brute_force():
    rng = np.random.default_rng(4)
    # ordinary pixels, pixels over a wide dynamic range with both signs, and
    # patches built so that z - m lands exactly halfway between two float32
    # values in float64 while the exact difference does not
    A = rng.uniform(0, 255, (40, 64))
    B = (np.ldexp(rng.uniform(1, 2, (40, 64)), rng.integers(-60, 10, (40, 64)))
         * rng.choice([-1.0, 1.0], (40, 64)))
    C = np.zeros((3, 64))
    C[:, 0] = 1.0
    C[:, 1] = 2.0 ** -19
    C[:, 2] = [2.0 ** -52, -(2.0 ** -52), 0.0]
    Z = np.concatenate([A, B, C]).astype(np.float32)
    got = lowp.dc_removed32(Z)
    want = _dc_removed_brute(Z)
    np.testing.assert_array_equal(got.view(np.uint32), want.view(np.uint32))
    # the engineered ties: 1 - 2^-6 - 2^-25 -/+ 2^-58 rounds away from the
    # even neighbour 63/64 in the first patch, to it in the second and third
    assert got[80, 0] == np.float32(1 - 2.0 ** -6 - 2.0 ** -24)
    assert got[81, 0] == np.float32(1 - 2.0 ** -6) == got[82, 0]


def test_dc_removed_order_free():
    # the definition names no summation order: permuting a patch's pixels
    # permutes its DC-removed values, and both modes share it
    rng = np.random.default_rng(5)
    Z = (rng.uniform(0, 255, (300, 64)) + rng.normal(0, 30, (300, 64))).astype(np.float32)
    zt = lowp.dc_removed32(Z, "bf16")
    np.testing.assert_array_equal(zt, lowp.dc_removed32(Z, "fp8"))
    for s in range(3):
        perm = np.random.default_rng(10 + s).permutation(64)
        np.testing.assert_array_equal(lowp.dc_removed32(Z[:, perm]), zt[:, perm])
    # and it is the exact difference within half a float32 ulp
    exact = Z.astype(np.float64) - Z.astype(np.float64).mean(1, keepdims=True)
    ulp = np.spacing(np.abs(zt)).astype(np.float64)
    assert np.all(np.abs(zt - exact) <= 0.5 * ulp + 1e-12 * np.abs(exact))


@pytest.mark.parametrize("mode", ["bf16", "fp8"])
def test_costs_exact_when_operands_are_representable(mode):
    # U_k a signed permutation and nu_kj = 4^n (nu^-1/2 a power of two);
    # the image 100 + 2 checker + stripes of period 4 (columns) and 2 (rows)
    # has, in every 8x8 patch, the mean 100 exactly and z~ in
    # {+-0.5, +-1.5, +-2.5, +-3.5}: every operand is exact in both formats,
    # so the costs are the float64 ones up to the float32 rounding of L_k
    rng = np.random.default_rng(5)
    K = 3
    U = np.zeros((K, 64, 64))
    for k in range(K):
        perm = rng.permutation(64)
        U[k, perm, np.arange(64)] = rng.choice([-1.0, 1.0], 64)
    beta = 1.0
    nu = 4.0 ** rng.integers(0, 4, (K, 64))
    nu[:, 0] = 1.0
    lam = nu - 1.0 / beta
    w = np.full(K, 1.0 / K)
    rr, cc = np.meshgrid(np.arange(12), np.arange(13), indexing="ij")
    x = (100.0 + 2.0 * (1 - 2 * ((rr + cc) % 2)) + 1.0 * (1 - 2 * ((cc // 2) % 2))
         + 0.5 * (1 - 2 * (rr % 2)))
    got = lowp.lowp_costs(x.astype(np.float32), U, lam, w, beta, mode)
    r, c = o.patch_corners(12, 13)
    Zt, m = o.remove_dc(o.extract(x, r, c))
    assert np.all(m == 100.0)
    _, nu2, _, L = o.eigen_terms(lam, w, beta)
    want = o.selection_costs(Zt, U, nu2, L) - L + L.astype(np.float32)
    np.testing.assert_allclose(got, want, rtol=1e-13, atol=0)


@pytest.mark.parametrize("mode,rel", [("bf16", 2.0 ** -8), ("fp8", 2.0 ** -4)])
def test_costs_within_rounding_bound(mode, rel):
    c = fs.config_c1()
    x = np.asarray(c["y"][:24, :24], np.float32)
    beta = 4.0 / c["sigma"] ** 2
    got = lowp.lowp_costs(x, c["U"], c["lam"], c["w"], beta, mode)
    r, cc = o.patch_corners(24, 24)
    Zt, _ = o.remove_dc(o.extract(x.astype(np.float64), r, cc))
    _, nu, _, L = o.eigen_terms(c["lam"], c["w"], beta)
    want = o.selection_costs(Zt, c["U"], nu, L)
    # |c~ - c| <= sum_p |u_p z_p| (2 rel + rel^2) per projection, rel the
    # unit roundoff of the format (half its step): bound the squares with it
    K = c["U"].shape[0]
    for k in range(K):
        Ut = c["U"][k] / np.sqrt(nu[k])[None, :]
        C = Zt @ Ut
        A = np.abs(Zt) @ np.abs(Ut)
        d = A * (2 * rel + rel * rel) + 1e-6
        bound = np.sum(2 * np.abs(C) * d + d * d, axis=1) + np.abs(L[k]) * 2 ** -23
        assert np.all(np.abs(got[:, k] - want[:, k]) <= bound)


# ---------------------------------------------------------------- flat tail

def _flat_exact_mixture():
    """Signed-permutation bases; beta = 1.  Components 0 and 1 have flat
    tails of 3 (nu_P = 4) after r_k kept eigenvalues 13/3 and 49/15, whose
    flat-tail scales sqrt(1/nu_P - 1/nu_j) are 1/4 and 1/8; component 2 has
    no tail (r = 64) and nu_kj = 4^n."""
    rng = np.random.default_rng(7)
    K = 3
    U = np.zeros((K, 64, 64))
    for k in range(K):
        perm = rng.permutation(64)
        U[k, perm, np.arange(64)] = rng.choice([-1.0, 1.0], 64)
    lam = np.empty((K, 64))
    rank = np.array([5, 12, 64])
    for k in range(2):
        r = rank[k]
        n1 = r // 2
        lam[k, :n1] = 13.0 / 3.0
        lam[k, n1:r] = 49.0 / 15.0
        lam[k, r:] = 3.0
    nu = np.sort(4.0 ** rng.integers(0, 4, 64))[::-1]
    nu[-1] = 1.0
    lam[2] = nu - 1.0
    w = np.array([0.5, 0.25, 0.25])
    return U, lam, w, rank


def _checker_stripes(h, w):
    rr, cc = np.meshgrid(np.arange(h), np.arange(w), indexing="ij")
    return (100.0 + 2.0 * (1 - 2 * ((rr + cc) % 2)) + 1.0 * (1 - 2 * ((cc // 2) % 2))
            + 0.5 * (1 - 2 * (rr % 2)))


@pytest.mark.parametrize("mode", ["bf16", "fp8"])
def test_flat_costs_exact_when_operands_are_representable(mode):
    """Sec. 3.1's rewritten cost from exactly representable operands equals
    the float64 flat-tail cost (oracle/flat_tail.py), up to the float32
    rounding of L_k: pins the sign and the 1/nu_P |z~|^2 term."""
    from oracle import flat_tail as ft
    U, lam, w, rank = _flat_exact_mixture()
    s = lowp.flat_scales(lam + 1.0, rank)
    assert np.all(np.isin(s[0, :5], [0.25, 0.125])) and np.all(s[0, 5:] == 0)
    x = _checker_stripes(12, 13)
    got = lowp.lowp_costs(x.astype(np.float32), U, lam, w, 1.0, mode, rank=rank)
    r, c = o.patch_corners(12, 13)
    Zt, m = o.remove_dc(o.extract(x, r, c))
    assert np.all(m == 100.0)
    _, _, _, L = o.eigen_terms(lam, w, 1.0)
    want = ft.flat_tail_costs(Zt, U, lam, rank, w, 1.0) - L + L.astype(np.float32)
    np.testing.assert_allclose(got, want, rtol=1e-13, atol=1e-11)


@pytest.mark.parametrize("mode", ["bf16", "fp8"])
def test_flat_costs_without_tail_are_the_plain_costs(mode):
    c = fs.config_c1()
    x = np.asarray(c["y"][:20, :20], np.float32)
    beta = 8.0 / c["sigma"] ** 2
    K = c["U"].shape[0]
    plain = lowp.lowp_costs(x, c["U"], c["lam"], c["w"], beta, mode)
    flat = lowp.lowp_costs(x, c["U"], c["lam"], c["w"], beta, mode, rank=np.full(K, 64))
    np.testing.assert_array_equal(flat, plain)


@pytest.mark.parametrize("mode,rel", [("bf16", 2.0 ** -8), ("fp8", 2.0 ** -4)])
def test_flat_costs_within_rounding_bound(mode, rel):
    """Rounded flat-tail costs stay within the operand-rounding bound of the
    exact flat-tail costs of the same spectra."""
    from oracle import flat_tail as ft
    c = fs.config_c1()
    lft, rank = ft.flat_tail(c["lam"], 0.95)
    assert rank.max() < 64
    x = np.asarray(c["y"][:24, :24], np.float32)
    beta = 4.0 / c["sigma"] ** 2
    got = lowp.lowp_costs(x, c["U"], lft, c["w"], beta, mode, rank=rank)
    r, cc = o.patch_corners(24, 24)
    Zt, _ = o.remove_dc(o.extract(x.astype(np.float64), r, cc))
    _, nu, _, L = o.eigen_terms(lft, c["w"], beta)
    want = ft.flat_tail_costs(Zt, c["U"], lft, rank, c["w"], beta)
    S = lowp.flat_scales(nu, rank)
    nz2 = np.sum(Zt * Zt, axis=1)
    for k in range(c["U"].shape[0]):
        Ut = c["U"][k] * S[k][None, :]
        C = Zt @ Ut
        A = np.abs(Zt) @ np.abs(Ut)
        d = A * (2 * rel + rel * rel) + 1e-6
        pinv = 1.0 / nu[k, rank[k]]
        bound = (np.sum(2 * np.abs(C) * d + d * d, axis=1) + np.abs(L[k]) * 2 ** -23
                 + pinv * nz2 * 2 ** -20)
        assert np.all(np.abs(got[:, k] - want[:, k]) <= bound)


# ---------------------------------------------------------------- estimation

def test_round_fp16_matches_torch():
    x = np.concatenate([_probe_values(11),
                        np.array([65504.0, 65519.0, 65520.0, 70000.0, 2.0 ** -24, 2.0 ** -25,
                                  3 * 2.0 ** -26, 1e-9, 0.0, -0.0], np.float32)])
    got = lowp.round_fp16(x)
    want = torch.from_numpy(x).to(torch.float16).to(torch.float64).numpy()
    np.testing.assert_array_equal(got, want)


def test_estimates_exact_when_operands_are_representable():
    # U_k a signed permutation, so W_k is diagonal (in permuted order) with
    # entries gamma_kj = lambda / (lambda + 1) at beta = 1; lambda in
    # {1, 3, 7, 15} makes them 1/2, 3/4, 7/8, 15/16, exact in binary16; the
    # checker-and-stripes image has mean 100 and z~ in {+-0.5, ..., +-3.5}
    rng = np.random.default_rng(13)
    K = 3
    U = np.zeros((K, 64, 64))
    for k in range(K):
        perm = rng.permutation(64)
        U[k, perm, np.arange(64)] = rng.choice([-1.0, 1.0], 64)
    lam = rng.choice([1.0, 3.0, 7.0, 15.0], (K, 64))
    w = np.full(K, 1.0 / K)
    x = _checker_stripes(12, 13).astype(np.float32)
    r, c = o.patch_corners(12, 13)
    lab = rng.integers(0, K, r.size)
    got = lowp.lowp_estimates(x, U, lam, w, 1.0, lab)
    Zt, m = o.remove_dc(o.extract(x.astype(np.float64), r, c))
    _, _, gamma, _ = o.eigen_terms(lam, w, 1.0)
    want = o.patch_estimate(Zt, m, lab, U, gamma)
    np.testing.assert_allclose(got, want, rtol=1e-14, atol=0)


def test_estimates_within_rounding_bound():
    c = fs.config_c1()
    x = np.asarray(c["y"][:20, :22], np.float32)
    beta = 8.0 / c["sigma"] ** 2
    r, cc = o.patch_corners(20, 22)
    lab = fs.rng(14).integers(0, c["U"].shape[0], r.size)
    got = lowp.lowp_estimates(x, c["U"], c["lam"], c["w"], beta, lab)
    Zt, m = o.remove_dc(o.extract(x.astype(np.float64), r, cc))
    _, _, gamma, _ = o.eigen_terms(c["lam"], c["w"], beta)
    want = o.patch_estimate(Zt, m, lab, c["U"], gamma)
    # W and z~ each rounded (float32, then binary16: relative 2^-11 + 2^-24)
    W = np.einsum("kqj,kj,kpj->kqp", c["U"], gamma, c["U"])
    u = 2.0 ** -11 + 2.0 ** -24
    mag = np.einsum("nqp,np->nq", np.abs(W[lab]), np.abs(Zt))
    assert np.all(np.abs(got - want) <= mag * (2 * u + u * u) + 1e-12)
    assert np.max(np.abs(got - want)) > 0  # (the rounding is there)
