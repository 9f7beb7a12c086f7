"""GPU cost-model network kernels against the float64 oracle (oracle/mlp_ref.py).

FP32 kernels vs float64 reference: forward outputs and every gradient entry
are compared with a relative tolerance sized for FP32 dot products of
length <= 64 (a few hundred ulp of the largest term); one Adam step is
compared elementwise; training on a fixed problem must reduce the loss.
"""
import numpy as np
import pytest

from oracle import mlp_ref
from paper_1306_4161_amd import hsumma as hs

pytestmark = pytest.mark.gpu

H = 64


def _pack(params):
    return np.concatenate([params[k].ravel() for k in ("W1", "b1", "W2", "b2", "W3", "b3")])


def _unpack(vec, F, K):
    out, o = {}, 0
    for k, shp in (("W1", (F, H)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("W3", (H, K)),
                   ("b3", (K,))):
        n = int(np.prod(shp))
        out[k] = vec[o:o + n].reshape(shp)
        o += n
    return out


def _problem(seed, N=48, F=11, K=9):
    r = np.random.default_rng(seed)
    X = r.normal(size=(N, F)).astype(np.float32).astype(np.float64)
    T = r.normal(size=(N, K)).astype(np.float32).astype(np.float64)
    mask = (r.uniform(size=(N, K)) < 0.7).astype(np.float64)
    params = mlp_ref.init(F, K, hidden=H, seed=seed)
    for k in ("b1", "b2", "b3"):
        params[k] = r.normal(scale=0.1, size=params[k].shape)
    params = {k: v.astype(np.float32).astype(np.float64) for k, v in params.items()}
    return params, X, T, mask


def _t(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda()


def test_forward_matches_oracle():
    params, X, T, mask = _problem(1)
    K = T.shape[1]
    Z = hs.mlp_forward(_t(X), _t(_pack(params)), H, K).cpu().numpy()
    Zr, _ = mlp_ref.forward(params, X)
    assert np.allclose(Z, Zr, rtol=1e-4, atol=1e-4 * np.abs(Zr).max())


def test_gradients_match_oracle():
    params, X, T, mask = _problem(2)
    F, K = X.shape[1], T.shape[1]
    loss, g, Z = hs.mlp_grad(_t(X), _t(T), _t(mask), _t(_pack(params)), H, K)
    g = _unpack(g.cpu().numpy().astype(np.float64), F, K)
    Zr, cache = mlp_ref.forward(params, X)
    gr = mlp_ref.backward(params, cache, Zr, T, mask)
    assert abs(float(loss.cpu()) - mlp_ref.loss(Zr, T, mask)) <= 1e-4 * mlp_ref.loss(Zr, T, mask)
    for k in gr:
        scale = np.abs(gr[k]).max() + 1e-12
        assert np.allclose(g[k], gr[k], rtol=2e-3, atol=2e-4 * scale), k


def test_adam_step_matches_oracle():
    import torch
    params, X, T, mask = _problem(3)
    F, K = X.shape[1], T.shape[1]
    p = _t(_pack(params))
    _, g, _ = hs.mlp_grad(_t(X), _t(T), _t(mask), p, H, K)
    gnp = g.cpu().numpy().astype(np.float64)
    m = torch.zeros_like(p)
    v = torch.zeros_like(p)
    before = p.cpu().numpy().astype(np.float64)
    hs.mlp_adam(p, g, m, v, 1, lr=1e-2)
    ref = {"x": before.copy()}
    mlp_ref.adam_step(ref, {"x": gnp}, {}, lr=1e-2)
    assert np.allclose(p.cpu().numpy(), ref["x"], rtol=1e-5, atol=1e-6)


def test_training_reduces_loss():
    import torch
    params, X, T, mask = _problem(4, N=256)
    F, K = X.shape[1], T.shape[1]
    p = _t(_pack(params))
    m = torch.zeros_like(p)
    v = torch.zeros_like(p)
    dX, dT, dm = _t(X), _t(T), _t(mask)
    l0 = float(hs.mlp_grad(dX, dT, dm, p, H, K)[0].cpu())
    for step in range(1, 301):
        _, g, _ = hs.mlp_grad(dX, dT, dm, p, H, K)
        hs.mlp_adam(p, g, m, v, step, lr=3e-3)
    l1 = float(hs.mlp_grad(dX, dT, dm, p, H, K)[0].cpu())
    assert l1 < 0.2 * l0
