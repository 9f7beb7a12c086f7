"""Autotuner and learned cost model on the GPU.

The tuner's optimum is pinned only by its own exhaustive search (parity
unpinned beyond that); what is checked: the chosen candidate is the fastest
timed one, the cache round-trips, disallowed candidates are never chosen,
and on held-out shapes the trained network's pick has lower runtime regret
than the untuned default configuration.
"""
import json
import os

import numpy as np
import pytest

from paper_1306_4161_amd import costmodel, tune

pytestmark = pytest.mark.gpu


def test_exhaustive_tune_and_cache(tmp_path):
    path = str(tmp_path / "cache.json")
    cache = tune.Cache(path)
    sh = tune.Shape(m=768, n=640, k=512, P=2, Q=2, G=4, M=128, sigma=0.0)
    name, opts = tune.tune(sh, cache, reps=2)
    times = cache.get(sh)["times"]
    assert name == min(times, key=times.get)
    assert set(times) == set(tune.NAMES)
    again = tune.Cache(path)
    assert again.get(sh)["best"] == name
    spread = tune.Shape(m=512, n=512, k=512, P=1, Q=1, G=1, M=128, sigma=4.0)
    name2, _ = tune.tune(spread, tune.Cache(str(tmp_path / "c2.json")), reps=1)
    assert not name2.startswith("split_")


def test_learned_model_beats_default_on_held_out_shapes():
    res = costmodel.experiment(n_shapes=90, seed=7, n_test=30, epochs=800, log=None,
                               lo=256, hi=4096)
    print(json.dumps({k: res[k] for k in ("regret_mlp", "regret_default", "best_static")}))
    assert res["regret_mlp"]["mean"] < res["regret_default"]["mean"]
    assert np.isfinite(res["regret_mlp"]["max"])


def test_groups_by_sampling_and_by_model():
    # the paper's procedure (Sec. V-A2): time a few HSUMMA iterations for
    # every valid G and keep the fastest; every G computes the same product
    res = tune.select_groups_by_sampling(1024, 4, 4, 32, 128, steps=2, reps=2)
    assert set(res["ms"]) == set(tune.valid_groups(4, 4)) == {1, 2, 4, 8, 16}
    assert res["G"] == min(res["ms"], key=res["ms"].get)
    assert all(t > 0 for t in res["ms"].values())
    m = tune.select_groups_by_model(1024, 4, 4, 32, 32, alpha=1e-4, beta=1e-9)
    assert m["G"] == 4 and m["sqrt_p_is_minimum"]        # eq. (11): sqrt(16) = 4
