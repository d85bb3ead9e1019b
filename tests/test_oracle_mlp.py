"""Pins of the proposal-network oracle (FP64): the forward map against
PyTorch's float64 linear and tanh-form GELU, gradients against central
finite differences, the first AdamW step against its closed form, the GELU
form's identities and its distance to x Phi(x), and the degenerate settings
of the proposal rule that must reduce to the plain full-K selection."""
import math

import numpy as np
import pytest

import fepll_synth as fs
from oracle import mlp64 as M


def small_params(seed=1, d=7, h=6, K=5):
    g = fs.rng(seed)
    return {"W1": g.normal(0, 0.5, (h, d)), "b1": g.normal(0, 0.1, h),
            "W2": g.normal(0, 0.5, (h, h)), "b2": g.normal(0, 0.1, h),
            "W3": g.normal(0, 0.5, (K, h)), "b3": g.normal(0, 0.1, K)}


def test_gradients_match_central_differences():
    p = small_params()
    g = fs.rng(2)
    X = g.normal(0, 1, (9, 7))
    t = g.integers(0, 5, 9)
    _, grad = M.loss_and_grad(p, X, t)
    h = 1e-6
    for name in M.NAMES:
        fd = np.zeros_like(p[name])
        for idx in np.ndindex(p[name].shape):
            keep = p[name][idx]
            p[name][idx] = keep + h
            lp = M.softmax_xent(M.forward(p, X)[0], t)[0]
            p[name][idx] = keep - h
            lm = M.softmax_xent(M.forward(p, X)[0], t)[0]
            p[name][idx] = keep
            fd[idx] = (lp - lm) / (2 * h)
        err = np.abs(fd - grad[name]).max() / max(1e-12, np.abs(fd).max())
        assert err < 1e-6, (name, err)


def test_full_size_gradient_spot_check():
    p = fs.mlp_init(200, 3)
    g = fs.rng(4)
    X = g.normal(0, 1, (16, 65))
    t = g.integers(0, 200, 16)
    _, grad = M.loss_and_grad(p, X, t)
    h = 1e-6
    for name, idx in [("W1", (3, 64)), ("b1", (17,)), ("W2", (100, 7)),
                      ("b2", (255,)), ("W3", (t[0], 5)), ("b3", (t[1],))]:
        keep = p[name][idx]
        p[name][idx] = keep + h
        lp = M.softmax_xent(M.forward(p, X)[0], t)[0]
        p[name][idx] = keep - h
        lm = M.softmax_xent(M.forward(p, X)[0], t)[0]
        p[name][idx] = keep
        fd = (lp - lm) / (2 * h)
        assert abs(fd - grad[name][idx]) <= 1e-6 * max(1e-3, abs(fd)), (name, fd, grad[name][idx])


def test_adamw_first_step_closed_form():
    """After one step from zero moments, m_hat = g and v_hat = g^2, so each
    parameter moves by lr * (g / (|g| + eps) + wd * p)."""
    p = small_params(5)
    p0 = {k: v.copy() for k, v in p.items()}
    g = {k: fs.rng(6 + i).normal(0, 1, v.shape) for i, (k, v) in enumerate(p.items())}
    m = {k: np.zeros_like(v) for k, v in p.items()}
    v = {k: np.zeros_like(x) for k, x in p.items()}
    lr, eps, wd = 0.01, 1e-8, 0.05
    M.adamw_step(p, g, m, v, 1, lr=lr, eps=eps, wd=wd)
    for k in M.NAMES:
        want = p0[k] - lr * (g[k] / (np.abs(g[k]) + eps) + wd * p0[k])
        np.testing.assert_allclose(p[k], want, rtol=1e-12, atol=1e-15)


def test_gelu_tanh_form():
    # the tanh form against PyTorch's own float64 implementation of it, its
    # odd-part identity gelu(x) - gelu(-x) = x (sigmoid(t) + sigmoid(-t) = 1),
    # its limits, its distance to the exact x Phi(x) (below 5e-4, Phi(1) =
    # 0.8413447460685429), and its derivative against central differences
    torch = pytest.importorskip("torch")
    x = np.linspace(-9, 9, 3601)
    want = torch.nn.functional.gelu(torch.from_numpy(x), approximate="tanh").numpy()
    np.testing.assert_allclose(M.gelu(x), want, rtol=1e-13, atol=1e-14)
    np.testing.assert_allclose(M.gelu(x) - M.gelu(-x), x, rtol=1e-13, atol=1e-14)
    np.testing.assert_allclose(M.gelu(np.array([30.0, -30.0, 0.0])), [30.0, 0.0, 0.0], atol=1e-30)
    exact = torch.nn.functional.gelu(torch.from_numpy(x)).numpy()
    assert np.max(np.abs(M.gelu(x) - exact)) < 5e-4
    assert abs(M.gelu(np.array([1.0]))[0] - 0.8413447460685429) < 5e-4
    xs = np.linspace(-4, 4, 17)
    fd = (M.gelu(xs + 1e-6) - M.gelu(xs - 1e-6)) / 2e-6
    np.testing.assert_allclose(M.gelu_grad(xs), fd, atol=1e-8)


def test_forward_against_torch_functional():
    # the oracle's forward map against an independent evaluation by PyTorch's
    # float64 CPU ops (linear layers and the tanh-form GELU)
    torch = pytest.importorskip("torch")
    F = torch.nn.functional
    K = 13
    p = dict(fs.mlp_init(K, 41))
    for i, k in enumerate(("b1", "b2", "b3")):
        p[k] = fs.rng(50 + i).normal(0, 0.3, p[k].shape)
    X = fs.rng(42).normal(0, 1, (300, 65))
    got, _ = M.forward(p, X)
    t = {k: torch.from_numpy(np.asarray(v, np.float64)) for k, v in p.items()}
    h = F.gelu(F.linear(torch.from_numpy(X), t["W1"], t["b1"]), approximate="tanh")
    h = F.gelu(F.linear(h, t["W2"], t["b2"]), approximate="tanh")
    want = F.linear(h, t["W3"], t["b3"]).numpy()
    np.testing.assert_allclose(got, want, rtol=1e-12, atol=1e-12)


def test_xent_uniform_logits_is_log_K():
    for K in (2, 7, 200):
        loss, g = M.softmax_xent(np.zeros((3, K)), np.array([0, 1, K - 1]))
        assert abs(loss - math.log(K)) < 1e-14
        np.testing.assert_allclose(g.sum(axis=1), 0, atol=1e-15)


def test_topm_ties_to_lower_index():
    lg = np.array([[1.0, 3.0, 3.0, 0.5, 3.0]])
    np.testing.assert_array_equal(M.topm(lg, 3), [[1, 2, 4]])


def test_proposal_degenerate_settings_give_full_argmin():
    g = fs.rng(9)
    costs = g.normal(0, 5, (50, 12))
    logits = g.normal(0, 1, (50, 12))
    full = np.argmin(costs, axis=1)
    lab, fb = M.propose_select(costs, M.topm(logits, 8), math.inf)
    np.testing.assert_array_equal(lab, full)
    assert fb.all()
    lab, _ = M.propose_select(costs, M.topm(logits, 12), 0.5)
    np.testing.assert_array_equal(lab, full)
    lab, fb = M.propose_select(costs, M.topm(logits, 3), -math.inf)
    assert not fb.any()
    cand = M.topm(logits, 3)
    want = cand[np.arange(50), np.argmin(np.take_along_axis(costs, cand, 1), 1)]
    np.testing.assert_array_equal(lab, want)
