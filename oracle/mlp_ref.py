"""Float64 reference of the small cost-model network -- TEST INFRASTRUCTURE.

The learned form predicts, for one problem shape, the log run time of every
candidate kernel configuration; the configuration with the smallest
prediction is chosen.  Network (all dense, row-major batches):

    H1 = relu(X W1 + b1)        X: (N, F), W1: (F, 64)
    H2 = relu(H1 W2 + b2)       W2: (64, 64)
    Z  = H2 W3 + b3             W3: (64, K), one output per candidate
    L  = sum(mask (Z - T)^2) / max(1, sum(mask))

(mask marks the candidates that were timed for a shape).  Gradients by the
chain rule; Adam (Kingma and Ba, 2015) with bias correction.

Pinned by tests/test_mlp_ref.py against central finite differences of the
loss (independent of the backward formulas) and against closed forms of a
single linear layer.
"""
from __future__ import annotations

import numpy as np


def init(F: int, K: int, hidden: int = 64, seed: int = 0):
    """He-uniform weights, zero biases (float64)."""
    r = np.random.default_rng(seed)

    def he(fan_in, fan_out):
        lim = np.sqrt(6.0 / fan_in)
        return r.uniform(-lim, lim, (fan_in, fan_out))

    return {"W1": he(F, hidden), "b1": np.zeros(hidden),
            "W2": he(hidden, hidden), "b2": np.zeros(hidden),
            "W3": he(hidden, K), "b3": np.zeros(K)}


def forward(params, X):
    X = np.asarray(X, dtype=np.float64)
    A1 = X @ params["W1"] + params["b1"]
    H1 = np.maximum(A1, 0.0)
    A2 = H1 @ params["W2"] + params["b2"]
    H2 = np.maximum(A2, 0.0)
    Z = H2 @ params["W3"] + params["b3"]
    return Z, {"X": X, "A1": A1, "H1": H1, "A2": A2, "H2": H2}


def loss(Z, T, mask):
    d = (Z - T) * mask
    return float(np.sum(d * d) / max(1.0, float(np.sum(mask))))


def backward(params, cache, Z, T, mask):
    cnt = max(1.0, float(np.sum(mask)))
    dZ = 2.0 * (Z - T) * mask / cnt
    g = {}
    g["W3"] = cache["H2"].T @ dZ
    g["b3"] = dZ.sum(axis=0)
    dH2 = dZ @ params["W3"].T
    dA2 = dH2 * (cache["A2"] > 0)
    g["W2"] = cache["H1"].T @ dA2
    g["b2"] = dA2.sum(axis=0)
    dH1 = dA2 @ params["W2"].T
    dA1 = dH1 * (cache["A1"] > 0)
    g["W1"] = cache["X"].T @ dA1
    g["b1"] = dA1.sum(axis=0)
    return g


def adam_step(params, grads, state, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update in place; state holds m, v and the step count t."""
    state["t"] = state.get("t", 0) + 1
    t = state["t"]
    for k in params:
        m = state.setdefault("m_" + k, np.zeros_like(params[k]))
        v = state.setdefault("v_" + k, np.zeros_like(params[k]))
        m[...] = b1 * m + (1 - b1) * grads[k]
        v[...] = b2 * v + (1 - b2) * grads[k] ** 2
        mh = m / (1 - b1 ** t)
        vh = v / (1 - b2 ** t)
        params[k] -= lr * mh / (np.sqrt(vh) + eps)


def finite_difference(params, X, T, mask, name, idx, h=1e-6):
    """Central difference of the loss w.r.t. one parameter entry."""
    p = {k: v.copy() for k, v in params.items()}
    p[name][idx] += h
    lp = loss(forward(p, X)[0], T, mask)
    p[name][idx] -= 2 * h
    lm = loss(forward(p, X)[0], T, mask)
    return (lp - lm) / (2 * h)
