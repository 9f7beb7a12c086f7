"""Learned cost model: an MLP that predicts the best kernel configuration.

Trained on the autotuner's own timings (tune.py).  Input: features of one
problem shape (sizes, grid, groups, outer block, value spread, work items
per macro-tile width).  Output: the predicted log2 run time of every
candidate configuration relative to the shape's mean; a new shape needs one
forward pass instead of an exhaustive search.  The pick is the single
configuration best on the training shapes unless the network predicts
another one faster by more than a margin, chosen on a validation fifth of
the training shapes (timing noise of a few per cent on short launches
exceeds many of the real differences, and an argmin over noisy predictions
picks needlessly away from a good default).  Exhaustive search stays the
fallback and the yardstick: regret = t(picked) / t(best) - 1.

Training and inference run in the library's own HIP kernels
(hsumma_mlp_grad / hsumma_mlp_adam / hsumma_mlp_forward); this module only
prepares arrays.

    python -m paper_1306_4161_amd.costmodel --shapes 2000 --out results.json
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np

from . import hsumma as hs
from . import tune

HIDDEN = 64


def features(shape) -> np.ndarray:
    """Feature vector of a shape (dict or tune.Shape): sizes, grid, groups,
    outer block, value spread, and for each macro-tile width t the number of
    work items of a t x t tiling and the fraction of their area that is
    inside C (ragged tiles waste the rest)."""
    s = shape if isinstance(shape, dict) else shape.__dict__
    m, n, k, P, Q, G, M = (float(s[x]) for x in ("m", "n", "k", "P", "Q", "G", "M"))
    l2 = math.log2
    tiles = []
    for t in (32, 64, 128, 256):
        items = P * Q * math.ceil(m / P / t) * math.ceil(n / Q / t)
        tiles += [l2(items), m * n / (items * t * t)]
    return np.array([
        l2(m), l2(n), l2(k), l2(M), l2(P), l2(Q), l2(G),
        l2(m / P), l2(n / Q), l2(m * n * M) / 3.0,
        s.get("sigma", 0.0), float(s.get("sigma", 0.0) > tune.SPLIT_MAX_SIGMA),
        l2(m / P) - l2(n / Q), (m / P) % 128 / 128.0, (n / Q) % 128 / 128.0,
    ] + tiles, dtype=np.float64)


def targets(rows):
    """(T, mask): log2 ms per candidate relative to the shape's mean over its
    timed candidates (the ranking is what the pick needs; the common scale
    of a shape would otherwise take most of the network's fit), 1 where
    timed."""
    K = len(tune.NAMES)
    T = np.zeros((len(rows), K))
    mask = np.zeros((len(rows), K))
    for i, r in enumerate(rows):
        for j, name in enumerate(tune.NAMES):
            if name in r["times"]:
                T[i, j] = math.log2(max(r["times"][name], 1e-4))
                mask[i, j] = 1.0
        if mask[i].any():
            T[i] = np.where(mask[i] > 0, T[i] - T[i][mask[i] > 0].mean(), 0.0)
    return T, mask


class CostModel:
    def __init__(self, F: int, K: int, seed: int = 0):
        import torch
        r = np.random.default_rng(seed)
        H = HIDDEN

        def he(fi, fo):
            lim = math.sqrt(6.0 / fi)
            return r.uniform(-lim, lim, (fi, fo))

        vec = np.concatenate([he(F, H).ravel(), np.zeros(H), he(H, H).ravel(), np.zeros(H),
                              he(H, K).ravel(), np.zeros(K)])
        self.F, self.K = F, K
        self.params = torch.from_numpy(vec.astype(np.float32)).cuda()
        self.mu = np.zeros(F)
        self.sd = np.ones(F)
        self.tmu = 0.0

    def _x(self, X):
        import torch
        return torch.from_numpy(((X - self.mu) / self.sd).astype(np.float32)).cuda()

    def fit(self, X, T, mask, epochs: int = 2000, lr: float = 2e-3, log=None):
        """Full-batch Adam on the masked MSE of (log time - mean)."""
        import torch
        self.mu = X.mean(0)
        self.sd = X.std(0) + 1e-6
        self.tmu = float((T * mask).sum() / max(1.0, mask.sum()))
        dX = self._x(X)
        dT = torch.from_numpy(((T - self.tmu) * mask).astype(np.float32)).cuda()
        dm = torch.from_numpy(mask.astype(np.float32)).cuda()
        m = torch.zeros_like(self.params)
        v = torch.zeros_like(self.params)
        grads = torch.empty_like(self.params)
        work = hs.mlp_work(X.shape[0], HIDDEN, self.K)
        history = []
        for step in range(1, epochs + 1):
            loss, _, _ = hs.mlp_grad(dX, dT, dm, self.params, HIDDEN, self.K, grads=grads,
                                     work=work)
            hs.mlp_adam(self.params, grads, m, v, step, lr=lr)
            if step == 1 or step % 200 == 0 or step == epochs:
                history.append((step, float(loss.cpu())))
                if log:
                    log("epoch %d loss %.4f" % history[-1])
        return history

    def predict(self, X) -> np.ndarray:
        Z = hs.mlp_forward(self._x(X), self.params, HIDDEN, self.K)
        return Z.cpu().numpy().astype(np.float64) + self.tmu

    def choose(self, X, shapes, fallback=None, margin: float = 0.0) -> list:
        """The candidate with the smallest predicted time; with a fallback
        (one name, or one per shape), that one unless the pick is predicted
        faster by more than `margin` (log2 units)."""
        Z = self.predict(X)
        out = []
        for i, sh in enumerate(shapes):
            s = sh if isinstance(sh, dict) else sh.__dict__
            shp = tune.Shape(**s)
            order = np.argsort(Z[i])
            pick = next(tune.NAMES[j] for j in order if tune.allowed(shp, tune.NAMES[j]))
            if fallback is not None:
                fb = fallback if isinstance(fallback, str) else fallback[i]
                jf, jp = tune.NAMES.index(fb), tune.NAMES.index(pick)
                if Z[i, jf] - Z[i, jp] <= margin:
                    pick = fb
            out.append(pick)
        return out


def regret(rows, picks) -> np.ndarray:
    """t(pick) / t(best) - 1 per row (inf if the pick was not timed)."""
    out = []
    for r, p in zip(rows, picks):
        t = r["times"]
        out.append(t[p] / min(t.values()) - 1.0 if p in t else float("inf"))
    return np.array(out)


def summarize(rg: np.ndarray) -> dict:
    return {"mean": float(np.mean(rg)), "median": float(np.median(rg)),
            "p90": float(np.quantile(rg, 0.9)), "max": float(np.max(rg)),
            "frac_optimal": float(np.mean(rg <= 1e-9))}


def experiment(n_shapes: int, seed: int, n_test: int = 200, epochs: int = 2000, log=print,
               lo: int = 512, hi: int = 16384, reps: int = 3):
    """Dataset -> train on n_shapes - n_test -> regret on the held-out shapes."""
    shapes = tune.random_shapes(n_shapes, seed, lo=lo, hi=hi)
    t0 = time.time()
    rows = tune.build_dataset(shapes, reps=reps, log=log)
    t_label = time.time() - t0
    X = np.stack([features(r["shape"]) for r in rows])
    T, mask = targets(rows)
    ntr = n_shapes - n_test
    # the training shapes: 80 % fit the network, 20 % choose the margin by
    # which a predicted gain must beat the library's own (untuned) choice
    nfit = max(1, int(0.8 * ntr))
    best_static = min(tune.NAMES, key=lambda nm: np.mean(regret(rows[:nfit], [nm] * nfit)))
    lib = [tune.library_default(r["shape"]) for r in rows]
    model = CostModel(X.shape[1], T.shape[1], seed=seed)
    hist = model.fit(X[:nfit], T[:nfit], mask[:nfit], epochs=epochs, log=log)
    val_rows = rows[nfit:ntr]
    margins = [0.0, 0.05, 0.1, 0.2, 0.3, 0.5, 0.75, 1.0, 1e9]
    val = {mg: float(np.mean(regret(val_rows, model.choose(X[nfit:ntr], [r["shape"] for r in val_rows],
                                                          lib[nfit:ntr], mg))))
           for mg in margins} if val_rows else {1e9: 0.0}
    margin = min(val, key=lambda mg: (val[mg], -mg))
    test_rows = rows[ntr:]
    t1 = time.time()
    picks = model.choose(X[ntr:], [r["shape"] for r in test_rows], lib[ntr:], margin)
    t_pred = time.time() - t1
    rg_mlp = regret(test_rows, picks)
    rg_argmin = regret(test_rows, model.choose(X[ntr:], [r["shape"] for r in test_rows]))
    # baselines: the library's own untuned choice (its fitted rule), a fixed
    # 128 x 128 configuration, and the single configuration best on the
    # training shapes
    rg_lib = regret(test_rows, lib[ntr:])
    rg_def = regret(test_rows, [tune.DEFAULT] * len(test_rows))
    rg_static = regret(test_rows, [best_static] * len(test_rows))
    exhaustive_ms = float(np.mean([sum(r["times"].values()) for r in test_rows]))
    return {
        "shapes": n_shapes, "train": ntr, "test": n_test, "seed": seed,
        "labeling_seconds": t_label, "loss_history": hist,
        "regret_mlp": summarize(rg_mlp), "regret_mlp_argmin": summarize(rg_argmin),
        "margin_log2": margin, "validation_regret_by_margin": val,
        "regret_library_default": summarize(rg_lib),
        "regret_fixed_default": summarize(rg_def),
        "regret_best_static": summarize(rg_static), "best_static": best_static,
        "prediction_seconds_per_shape": t_pred / max(1, n_test),
        "exhaustive_timed_ms_per_shape": exhaustive_ms,
        "pick_histogram": {nm: picks.count(nm) for nm in set(picks)},
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--shapes", type=int, default=2000)
    ap.add_argument("--test", type=int, default=200)
    ap.add_argument("--seed", type=int, default=1306)
    ap.add_argument("--epochs", type=int, default=2000)
    ap.add_argument("--out", type=str, default="")
    a = ap.parse_args()

    def log(msg):
        print("[costmodel] " + msg, file=sys.stderr, flush=True)

    res = experiment(a.shapes, a.seed, a.test, a.epochs, log=log)
    txt = json.dumps(res, indent=1)
    print(txt)
    if a.out:
        with open(a.out, "w") as f:
            f.write(txt)


if __name__ == "__main__":
    main()
