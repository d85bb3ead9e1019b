"""Reduced-precision Gaussian selection -- the reference definitions.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
benchmark's CPU-baseline leg may import this module; the restoration library
never does, and this module imports nothing from it.

The paper evaluates the selection cost of Alg. 1 (Gaussian selection, in the
eigenspace form of Sec. 2.1) in full precision.  The library also offers two
reduced-precision selection modes -- a builder's choice, not the paper's --
in which the projections c = Ut_k^t z~, Ut_k = U_k diag(nu_k)^-1/2, take
rounded operands:

* ``"bf16"``: z~ and Ut_k rounded to bfloat16 (8 significant bits, nearest,
  ties to even);
* ``"fp8"``:  z~ and Ut_k scaled by powers of two, 2^-e_z per patch and
  2^-e_k per component, e the smallest integer that brings the largest
  magnitude to at most 448, then rounded to e4m3 (OCP "E4M3FN": 4 exponent
  bits with bias 7, 3 mantissa bits, subnormal step 2^-9, largest finite 448,
  no infinities; nearest, ties to even); the scales are applied back
  exactly.

The patch estimate of Alg. 1 in these modes (``lowp_estimates``) takes
binary16 operands: W_k = U_k diag(gamma_k) U_k^t formed in float64, rounded
to float32 and then to binary16 (11 significant bits, nearest, ties to
even), and the float32 DC-removed patch rounded to binary16; the estimate is
W16 z16 + m with exact products and the patch mean m of the DC removal.

In both modes the cost is L_k + sum_j c_j^2 with L_k rounded from float64 to
float32, and the products are exact: this module evaluates them in float64
from the rounded operands.  What the GPU adds on top is float32 (or wider)
accumulation, so its costs must agree with these to within that rounding.

The DC-removed patch z~ is defined independently of any summation order: m
is the sum of the patch's 64 float32 pixels, correctly rounded to float64
(exact whenever the pixel magnitudes of the patch lie within a factor 2^23
of each other), divided by 64 (exact), and each z~_j is the difference
z_j - m correctly rounded to float32 (nearest, ties to even).  Both modes
share it, and it is the float32 path's DC removal too.

Ut_k is formed in float64 and rounded to float32 before the format rounding
(for fp8: Ut_k 2^-e_k rounded to float32, then to e4m3).

Flat-tail form (Sec. 3.1, ``rank`` given, lam the flat-tailed spectra):
for a component with r_k < 64 kept eigenvalues, Sec. 3.1's rewritten cost

  L_k + |z~|^2 / nu_P - sum_{j < r_k} c_j^2 (1/nu_P - 1/nu_j)

is evaluated with the operand Ut_k = U_k diag(s), s_j = sqrt(1/nu_P - 1/nu_j)
for j < r_k and 0 beyond (nu_P the tail's nu), rounded as above; 1/nu_P is
rounded from float64 to float32, and |z~|^2 is the exact squared norm of the
float32 DC-removed patch (before the format rounding).  Components with
r_k = 64 keep the plain form.
"""
from __future__ import annotations

import math

import numpy as np

from . import epll64 as o

E4M3_MAX = 448.0


# ----------------------------------------------------------- rounding

def round_bf16(x) -> np.ndarray:
    """Nearest bfloat16 value (ties to even) of float32 x, as float32.

    bfloat16 keeps float32's exponent range and 8 significant bits: on the
    binade [2^(e-1), 2^e) the step is 2^(e-8), and below 2^-126 the step is
    the smallest bfloat16 subnormal, 2^-133."""
    x = np.asarray(x, np.float32).astype(np.float64)
    _, e = np.frexp(x)
    step = np.ldexp(1.0, np.maximum(e - 8, -133))
    r = np.rint(x / step) * step  # rint: nearest, ties to even
    return r.astype(np.float32)


def round_fp16(x) -> np.ndarray:
    """Nearest IEEE binary16 value (ties to even) of float32 x, in float64;
    +-inf where the rounded magnitude exceeds 65504.

    binary16 keeps 11 significant bits: on the binade [2^(e-1), 2^e),
    e - 1 >= -14, the step is 2^(e-11); below 2^-14 the subnormal step is
    2^-24."""
    x = np.asarray(x, np.float32).astype(np.float64)
    _, e = np.frexp(x)
    step = np.ldexp(1.0, np.maximum(e - 11, -24))
    r = np.rint(x / step) * step
    return np.where(np.abs(r) > 65504.0, np.copysign(np.inf, r), r)


def round_e4m3(x) -> np.ndarray:
    """Nearest e4m3 value (ties to even) of x, in float64; NaN where the
    rounded magnitude exceeds 448 (the format has no infinity and the
    conversion does not saturate).

    Normal binades [2^(e-1), 2^e) for e - 1 >= -6 have the step 2^(e-4)
    (3 mantissa bits); below 2^-6 the subnormal step is 2^-9."""
    x = np.asarray(x, np.float64)
    _, e = np.frexp(x)
    step = np.ldexp(1.0, np.maximum(e - 4, -9))
    r = np.rint(x / step) * step
    return np.where(np.abs(r) > E4M3_MAX, np.nan, r)


def pow2_exponent(mx) -> np.ndarray:
    """Smallest integer e with mx * 2^-e <= 448 (0 for mx = 0), at least -127."""
    mx = np.asarray(mx, np.float64)
    out = np.zeros(mx.shape, np.int64)
    pos = mx > 0
    e = np.ceil(np.log2(np.where(pos, mx, 1.0) / E4M3_MAX)).astype(np.int64)
    # settle the float log2 exactly: mx 2^-e <= 448 < mx 2^-(e-1)
    for _ in range(2):
        e = np.where(np.ldexp(mx, -e) > E4M3_MAX, e + 1, e)
        e = np.where(np.ldexp(mx, -(e - 1)) <= E4M3_MAX, e - 1, e)
    out[pos] = e[pos]
    return np.maximum(out, -127)


# ----------------------------------------------------------- operands

def _twosum(a: np.ndarray, b: np.ndarray):
    """s + e == a + b exactly, s = fl(a + b) (Knuth's TwoSum)."""
    s = a + b
    bv = s - a
    av = s - bv
    return s, (a - av) + (b - bv)


def round32_of_sum(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """a + b (float64 arrays) correctly rounded to float32, nearest, ties to
    even: the float64 sum d and its error e give the exact value d + e;
    rounding d alone is correct unless d sits exactly halfway between two
    float32 values and e != 0, where e decides."""
    d, e = _twosum(np.asarray(a, np.float64), np.asarray(b, np.float64))
    r = d.astype(np.float32)
    r64 = r.astype(np.float64)
    # the other float32 neighbour of d (toward d), and the midpoint between
    # the two (exact in float64)
    nb = np.nextafter(r, np.where(d > r64, np.inf, -np.inf).astype(np.float32))
    nb64 = nb.astype(np.float64)
    mid = (r64 + nb64) * 0.5
    # a tie of d went to the even neighbour r; the exact value d + e lies
    # past the midpoint, toward nb, when e points that way
    fix = (e != 0) & (d == mid) & ((e > 0) == (nb64 > r64))
    return np.where(fix, nb, r)


def dc_removed32(Z: np.ndarray, mode: str | None = None) -> np.ndarray:
    """z~ = z - m in float32 for float32 patches Z (N x 64), m as in the
    module docstring (the same for both modes)."""
    Z64 = np.asarray(Z, np.float32).astype(np.float64)
    S = np.fromiter((math.fsum(row) for row in Z64), np.float64, Z64.shape[0])
    m = S * (1.0 / 64.0)
    return round32_of_sum(Z64, -m[:, None])


def patch_operand(Zt32: np.ndarray, mode: str) -> np.ndarray:
    """The rounded patch operand (N x 64, float64 values, scale applied)."""
    if mode == "bf16":
        return round_bf16(Zt32).astype(np.float64)
    e = pow2_exponent(np.max(np.abs(Zt32.astype(np.float64)), axis=1))
    q = round_e4m3(np.ldexp(Zt32.astype(np.float64), -e[:, None]))
    return np.ldexp(q, e[:, None])


def flat_scales(nu: np.ndarray, rank) -> np.ndarray:
    """Column scales of the flat-tail operand (K x 64): sqrt(1/nu_P - 1/nu_j)
    for the kept directions, 0 for the tail; 1/sqrt(nu_j) for components
    without a tail."""
    nu = np.asarray(nu, np.float64)
    K, P = nu.shape
    s = np.zeros((K, P))
    for k in range(K):
        rk = int(rank[k])
        if rk >= P:
            s[k] = 1.0 / np.sqrt(nu[k])
        else:
            s[k, :rk] = np.sqrt(np.maximum(1.0 / nu[k, rk] - 1.0 / nu[k, :rk], 0.0))
    return s


def basis_operand(U: np.ndarray, nu: np.ndarray, mode: str, rank=None) -> np.ndarray:
    """The rounded Ut_k = U_k diag(nu_k)^-1/2 (K x 64 x 64, float64 values,
    scale applied); with ``rank``, the flat-tail operand U_k diag(s)."""
    if rank is None:
        Ut = np.asarray(U, np.float64) / np.sqrt(nu)[:, None, :]
    else:
        Ut = np.asarray(U, np.float64) * flat_scales(nu, rank)[:, None, :]
    if mode == "bf16":
        return round_bf16(Ut.astype(np.float32)).astype(np.float64)
    e = pow2_exponent(np.max(np.abs(Ut), axis=(1, 2)))
    q = round_e4m3(np.ldexp(Ut, -e[:, None, None]).astype(np.float32).astype(np.float64))
    return np.ldexp(q, e[:, None, None])


# ----------------------------------------------------------- selection

def lowp_costs(x, U, lam, w, beta, mode: str, acc_eps: float | None = None, rank=None,
               patches=None):
    """Selection costs (Np x K, float64) of every valid patch of the float32
    image x in a reduced-precision mode: float32(L_k) + sum_j c_j^2 with c
    the exact product of the rounded operands.  With ``rank`` (lam then the
    flat-tailed spectra), the flat-tail form of the module docstring.

    With ``acc_eps``, also return a bound (Np x K) on how far an evaluation
    may land from these costs when it accumulates each projection c_j with a
    relative error of at most acc_eps of sum_p |Ut[p,j] z[p]| and the 64
    squares, |z~|^2, and the terms of the cost in float32.

    ``patches``: indices (r (W - 7) + c) of the valid patches to evaluate
    (default: all, in that order)."""
    x = np.asarray(x, np.float32)
    H, W = x.shape
    r, c = o.patch_corners(H, W)
    if patches is not None:
        r, c = r[patches], c[patches]
    Z = o.extract(x.astype(np.float64), r, c).astype(np.float32)  # exact: x is float32
    Zt32 = dc_removed32(Z, mode)
    Zq = patch_operand(Zt32, mode)
    _, nu, _, L = o.eigen_terms(np.asarray(lam, np.float64), np.asarray(w, np.float64), beta)
    Uq = basis_operand(U, nu, mode, rank)
    L32 = L.astype(np.float32).astype(np.float64)
    K, P = Uq.shape[0], Uq.shape[1]
    if rank is not None:
        z64 = Zt32.astype(np.float64)
        nz2 = np.sum(z64 * z64, axis=1)
    cost = np.empty((Zq.shape[0], K))
    bound = np.empty_like(cost) if acc_eps is not None else None
    u32 = 2.0 ** -24
    for k in range(K):
        C = Zq @ Uq[k]
        sq = np.sum(C * C, axis=1)
        flat = rank is not None and int(rank[k]) < P
        if flat:
            pinv = float(np.float32(1.0 / nu[k, int(rank[k])]))
            cost[:, k] = L32[k] + pinv * nz2 - sq
        else:
            cost[:, k] = L32[k] + sq
        if bound is not None:
            d = acc_eps * (np.abs(Zq) @ np.abs(Uq[k]))
            # flat tail: |z~|^2 summed in float32 (64 roundings), then
            # two more roundings of the cost's terms
            bound[:, k] = (np.sum(2 * np.abs(C) * d + d * d, axis=1)
                           + 65 * u32 * (sq + np.abs(L32[k]))
                           + (130 * u32 * pinv * nz2 if flat else 0.0))
    return (cost, bound) if bound is not None else cost


# ----------------------------------------------------------- estimation

def estimate_operand(U, lam, w, beta) -> np.ndarray:
    """The binary16 Wiener operand W_k = U_k diag(gamma_k) U_k^t (K x 64 x
    64, float64 values): formed in float64, rounded to float32, then to
    binary16."""
    _, _, gamma, _ = o.eigen_terms(np.asarray(lam, np.float64), np.asarray(w, np.float64), beta)
    U = np.asarray(U, np.float64)
    W = np.einsum("kqj,kj,kpj->kqp", U, gamma, U)
    return round_fp16(W.astype(np.float32))


def lowp_estimates(x, U, lam, w, beta, labels, acc_eps: float | None = None, patches=None):
    """Patch estimates (N x 64, float64) of the float32 image x under the
    given labels in the reduced-precision modes: z^ = W16_k z16 + m, W16 of
    ``estimate_operand``, z16 the binary16 rounding of the float32 DC-removed
    patch, m its mean (the sum of the pixels correctly rounded to float64,
    divided by 64), products exact.

    With ``acc_eps``, also a bound (N x 64) on how far an evaluation may land
    from these estimates when it accumulates the 64 products with a relative
    error of at most acc_eps of the sum of their magnitudes, adds m rounded
    to float32 and rounds the sum to float32.

    ``patches``: indices (r (W - 7) + c) of the valid patches (default: all,
    in that order); labels holds one entry per patch evaluated."""
    x = np.asarray(x, np.float32)
    H, W = x.shape
    r, c = o.patch_corners(H, W)
    if patches is not None:
        r, c = r[patches], c[patches]
    Z = o.extract(x.astype(np.float64), r, c).astype(np.float32)
    Z64 = Z.astype(np.float64)
    S = np.fromiter((math.fsum(row) for row in Z64), np.float64, Z64.shape[0])
    m = S * (1.0 / 64.0)
    z16 = round_fp16(round32_of_sum(Z64, -m[:, None]))
    W16 = estimate_operand(U, lam, w, beta)
    lab = np.asarray(labels, np.int64)
    prod = np.einsum("nqp,np->nq", W16[lab], z16)
    est = prod + m[:, None]
    if acc_eps is None:
        return est
    mag = np.einsum("nqp,np->nq", np.abs(W16[lab]), np.abs(z16))
    u32 = 2.0 ** -24
    bound = acc_eps * mag + u32 * np.abs(m)[:, None] + u32 * (np.abs(est) + acc_eps * mag)
    return est, bound
