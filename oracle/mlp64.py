"""FP64 CPU reference of the component-proposal network -- oracle side.

TEST INFRASTRUCTURE ONLY (imported by tests, the smoke check and the
benchmark's CPU-baseline leg, never by the restoration library).

The paper does not use a network for the Gaussian selection step: it reviews
a gating network (Sec. 4, Related methods, its RoG score) that approximates
the selection score, and accelerates the step with a search tree instead.
The proposal network here is a design choice of this project that takes the
same role -- guess the few components worth scoring -- and is then checked by
the exact score of the selection step (Eq. (8)), so the
restoration stays the paper's method.  Everything below is therefore
defined by this project, not by the paper:

* input feature of a patch: [z~ / 128, log sigma_beta] (65 values), with z~
  the DC-removed patch and sigma_beta = beta^-1/2;
* network: 65 -> 256 -> 256 -> K, GELU in its tanh form (Hendrycks &
  Gimpel, 2016) after the two hidden layers, logits out;  h = W x + b with W stored (out, in) row-major;
* loss: mean softmax cross-entropy against the MAP label k*;
* optimiser: AdamW with decoupled weight decay
  p <- p - lr * (m_hat / (sqrt(v_hat) + eps) + wd * p), bias-corrected moments;
* proposal: the top-m logits (ties: lower index), exact costs for those m
  components, the best of them (ties: lower index); if half the gap between
  the two best exact costs is below ``margin`` nats the patch takes the
  full-K argmin instead.
"""
from __future__ import annotations

import math

import numpy as np

SCALE_IN = 128.0
NAMES = ("W1", "b1", "W2", "b2", "W3", "b3")


def features(Zt: np.ndarray, beta: float) -> np.ndarray:
    """[z~/128, log sigma_beta] per patch, sigma_beta = beta^-1/2."""
    n = Zt.shape[0]
    f = np.empty((n, Zt.shape[1] + 1))
    f[:, :-1] = Zt / SCALE_IN
    f[:, -1] = -0.5 * math.log(beta)
    return f


def gelu(x):
    """x * sigmoid(2 u) = 0.5 x (1 + tanh u), u = sqrt(2/pi) (x + 0.044715 x^3)."""
    u = math.sqrt(2.0 / math.pi) * (x + 0.044715 * x ** 3)
    return 0.5 * x * (1.0 + np.tanh(u))


def gelu_grad(x):
    """Derivative of ``gelu`` by the chain rule."""
    t = np.tanh(math.sqrt(2.0 / math.pi) * (x + 0.044715 * x ** 3))
    du = math.sqrt(2.0 / math.pi) * (1.0 + 3.0 * 0.044715 * x * x)
    return 0.5 * (1.0 + t) + 0.5 * x * (1.0 - t * t) * du


def forward(p, X):
    """Returns logits and the activations needed by ``backward``."""
    a1 = X @ p["W1"].T + p["b1"]
    h1 = gelu(a1)
    a2 = h1 @ p["W2"].T + p["b2"]
    h2 = gelu(a2)
    logits = h2 @ p["W3"].T + p["b3"]
    return logits, (X, a1, h1, a2, h2)


def softmax_xent(logits, target):
    """Mean cross-entropy and its gradient w.r.t. the logits."""
    n = logits.shape[0]
    z = logits - logits.max(axis=1, keepdims=True)
    lse = np.log(np.exp(z).sum(axis=1))
    loss = float(np.mean(lse - z[np.arange(n), target]))
    g = np.exp(z - lse[:, None])
    g[np.arange(n), target] -= 1.0
    return loss, g / n


def backward(p, cache, dlogits):
    """Gradients of all parameters by the chain rule."""
    X, a1, h1, a2, h2 = cache
    g = {}
    g["W3"] = dlogits.T @ h2
    g["b3"] = dlogits.sum(axis=0)
    dh2 = dlogits @ p["W3"]
    da2 = dh2 * gelu_grad(a2)
    g["W2"] = da2.T @ h1
    g["b2"] = da2.sum(axis=0)
    dh1 = da2 @ p["W2"]
    da1 = dh1 * gelu_grad(a1)
    g["W1"] = da1.T @ X
    g["b1"] = da1.sum(axis=0)
    return g


def loss_and_grad(p, X, target):
    logits, cache = forward(p, X)
    loss, dl = softmax_xent(logits, target)
    return loss, backward(p, cache, dl)


def adamw_step(p, g, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8, wd=1e-4):
    """One AdamW update in place (t counts from 1)."""
    for k in NAMES:
        m[k] = b1 * m[k] + (1.0 - b1) * g[k]
        v[k] = b2 * v[k] + (1.0 - b2) * g[k] * g[k]
        mh = m[k] / (1.0 - b1 ** t)
        vh = v[k] / (1.0 - b2 ** t)
        p[k] = p[k] - lr * (mh / (np.sqrt(vh) + eps) + wd * p[k])


def topm(logits: np.ndarray, m: int) -> np.ndarray:
    """Indices of the m largest logits per row, ties to the lower index."""
    order = np.argsort(-logits, axis=1, kind="stable")
    return order[:, :m]


def propose_select(costs: np.ndarray, cand: np.ndarray, margin: float):
    """Label of the proposal path from exact costs (n, K) and candidate
    sets (n, m): best candidate, or the full-K argmin when half the exact
    gap between the two best candidates is below ``margin`` nats.
    Returns (labels, fell_back)."""
    n = costs.shape[0]
    cc = np.take_along_axis(costs, cand, axis=1)
    # order candidates by (cost, index) so ties go to the lower index
    order = np.lexsort((cand, cc), axis=1) if cand.shape[1] > 1 else np.zeros_like(cand)
    c_sorted = np.take_along_axis(cc, order, axis=1)
    k_sorted = np.take_along_axis(cand, order, axis=1)
    lab = k_sorted[:, 0].copy()
    if cand.shape[1] > 1:
        gap = 0.5 * (c_sorted[:, 1] - c_sorted[:, 0])
    else:
        gap = np.full(n, -np.inf)
    fb = ~(gap >= margin)
    full = np.argmin(costs, axis=1)
    lab[fb] = full[fb]
    return lab, fb
