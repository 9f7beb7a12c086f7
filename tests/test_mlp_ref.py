"""Pins of the float64 cost-model network reference (oracle/mlp_ref.py)."""
import numpy as np

from oracle import mlp_ref


def _problem(seed=0, N=12, F=7, K=5):
    r = np.random.default_rng(seed)
    X = r.normal(size=(N, F))
    T = r.normal(size=(N, K))
    mask = (r.uniform(size=(N, K)) < 0.8).astype(np.float64)
    params = mlp_ref.init(F, K, hidden=64, seed=seed + 1)
    for k in ("b1", "b2", "b3"):
        params[k] = r.normal(scale=0.1, size=params[k].shape)
    return params, X, T, mask


def test_backward_matches_central_differences():
    params, X, T, mask = _problem()
    Z, cache = mlp_ref.forward(params, X)
    g = mlp_ref.backward(params, cache, Z, T, mask)
    r = np.random.default_rng(5)
    for name in params:
        for _ in range(6):
            idx = tuple(int(r.integers(0, s)) for s in params[name].shape)
            fd = mlp_ref.finite_difference(params, X, T, mask, name, idx)
            assert abs(fd - g[name][idx]) <= 1e-6 * max(1.0, abs(fd)), (name, idx, fd, g[name][idx])


def test_single_linear_layer_closed_form():
    # with relu layers bypassed (identity weights, positive activations) the
    # output gradient of a linear least-squares layer is 2 H^T (Z - T) / count
    r = np.random.default_rng(3)
    N, K = 9, 4
    params = mlp_ref.init(64, K, seed=2)
    params["W1"] = np.eye(64); params["W2"] = np.eye(64)
    params["b1"][:] = 0; params["b2"][:] = 0
    X = np.abs(r.normal(size=(N, 64))) + 0.1
    T = r.normal(size=(N, K))
    mask = np.ones((N, K))
    Z, cache = mlp_ref.forward(params, X)
    assert np.allclose(Z, X @ params["W3"] + params["b3"])
    g = mlp_ref.backward(params, cache, Z, T, mask)
    assert np.allclose(g["W3"], 2 * X.T @ (Z - T) / (N * K))
    assert np.allclose(g["b3"], 2 * (Z - T).sum(0) / (N * K))


def test_adam_first_step_is_signed_lr():
    # Adam's bias-corrected first step is lr * g / (|g| + eps): ~lr * sign(g)
    params, X, T, mask = _problem(seed=4)
    Z, cache = mlp_ref.forward(params, X)
    g = mlp_ref.backward(params, cache, Z, T, mask)
    before = {k: v.copy() for k, v in params.items()}
    mlp_ref.adam_step(params, g, {}, lr=1e-3, eps=1e-8)
    for k in params:
        step = params[k] - before[k]
        expect = -1e-3 * g[k] / (np.abs(g[k]) + 1e-8)
        assert np.allclose(step, expect, rtol=1e-9, atol=1e-15)


def test_training_reduces_loss():
    params, X, T, mask = _problem(seed=7, N=64)
    state = {}
    l0 = mlp_ref.loss(mlp_ref.forward(params, X)[0], T, mask)
    for _ in range(300):
        Z, cache = mlp_ref.forward(params, X)
        mlp_ref.adam_step(params, mlp_ref.backward(params, cache, Z, T, mask), state, lr=3e-3)
    l1 = mlp_ref.loss(mlp_ref.forward(params, X)[0], T, mask)
    assert l1 < 0.2 * l0
