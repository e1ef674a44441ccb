"""Autotuner logic on the CPU (search, rejection, cache) with a synthetic
cost; the GPU test runs it on a real build and checks that the chosen
options leave the results unchanged."""
import json
import os

import numpy as np
import pytest

from paper_1610_05266_amd import tune


def test_coordinate_search_finds_the_best_values_and_respects_noise():
    target = {"bin_scale": 1.5, "fast_radius": 3.0, "closure_radius": 4.5, "region_h": 4.0}

    def cost(o):
        return 1.0 + sum((o[k] - target[k]) ** 2 for k in target)

    res = tune.coordinate_search(cost)
    for k in target:
        assert res.options[k] == target[k]
    assert res.median_ms == pytest.approx(1.0)
    assert res.default_ms == cost(tune.DEFAULTS)
    # a gain below the noise margin is not taken
    res2 = tune.coordinate_search(lambda o: 1.0 - 0.001 * o["bin_scale"])
    assert res2.options == tune.DEFAULTS


def test_rejected_candidates_are_skipped():
    def cost(o):
        if o["fast_radius"] > 2.9:
            return None          # e.g. a result that changed, or a failed build
        return 10.0 - o["fast_radius"]

    res = tune.coordinate_search(cost)
    assert res.options["fast_radius"] == 2.8
    assert any(t["ms"] is None for t in res.trials)
    with pytest.raises(RuntimeError):
        tune.coordinate_search(lambda o: None)


def test_cache_round_trip_and_keys(tmp_path):
    p = str(tmp_path / "sub" / "t.json")
    tune._store(p, {"k": {"options": tune.DEFAULTS, "median_ms": 1.0, "default_ms": 2.0}})
    assert tune._load(p)["k"]["median_ms"] == 1.0
    assert tune._load(str(tmp_path / "missing.json")) == {}
    k1 = tune.workload_key("gfx950", 1_048_576, 66049, 0.25, 1)
    k2 = tune.workload_key("gfx950", 1_050_000, 66100, 0.25, 1)
    k3 = tune.workload_key("gfx950", 4_194_304, 263169, 0.25, 1)
    assert k1 == k2 and k1 != k3
    os.environ[tune.CACHE_ENV] = p
    try:
        assert tune.default_cache_path() == p
    finally:
        del os.environ[tune.CACHE_ENV]


def test_choose_takes_the_fastest_equal_variant(tmp_path):
    """The variant chooser on the CPU: a synthetic cost per variant, one
    variant whose result differs (rejected however fast), the noise margin,
    and the cache."""
    import torch

    state = {"v": "a"}
    cost = {"a": 1.0, "b": 0.7, "c": 0.5, "d": 0.995}
    out = torch.zeros(4)

    def run():
        out.fill_(1.0 if state["v"] != "c" else 2.0)   # "c" computes something else

    variants = {k: (lambda k=k: state.__setitem__("v", k)) for k in ("a", "b", "c", "d")}
    path = str(tmp_path / "choose.json")
    res = tune.choose(variants, run, lambda: [out], "k1", cache_path=path, time_of=lambda fn: cost[state["v"]])
    assert res["choice"] == "b" and not res["cached"] and state["v"] == "b"
    assert res["ms"] == pytest.approx(0.7) and res["default_ms"] == pytest.approx(1.0)
    # a gain inside the noise margin keeps the default
    only = {k: variants[k] for k in ("a", "d")}
    assert tune.choose(only, run, lambda: [out], "k2", cache_path=path,
                       time_of=lambda fn: cost[state["v"]])["choice"] == "a"
    # the cache answers without timing, and selects the cached variant
    state["v"] = "a"
    again = tune.choose(variants, run, lambda: [out], "k1", cache_path=path, time_of=None)
    assert again["cached"] and again["choice"] == "b" and state["v"] == "b"
    assert set(tune.m2p_variants()) == {"m2p_ppt=1", "m2p_ppt=2", "m2p_ppt=4"}


@pytest.mark.gpu
def test_autotune_on_gpu_keeps_results_and_uses_the_cache(tmp_path):
    import torch

    import workloads as wl
    from paper_1610_05266_amd import ops
    from paper_1610_05266_amd._lib import P2M_WEIGHTS_F32

    c = wl.small_cloud(64, 4, 0.3, seed=3, channels=("u", "v", "q"))
    pos = torch.from_numpy(c.pos).cuda()
    vals = torch.from_numpy(c.vals).cuda()
    w = ops.Weights()

    def build():
        return ops.p2m_build_weights(c.mesh, c.h, pos, P2M_WEIGHTS_F32, weights=w, check_diag=False)

    def probe(h):
        return ops.p2m_project(h, vals)

    path = str(tmp_path / "tune.json")
    try:
        res = tune.autotune(build, probe, "test-key", cache_path=path, repeats=3)
        assert not res.cached and res.median_ms <= res.default_ms
        tuned = probe(build()).clone()
        tune.apply_options(tune.DEFAULTS)
        assert torch.equal(tuned, probe(build()))
        again = tune.autotune(build, probe, "test-key", cache_path=path)
        assert again.cached and again.options == res.options
        assert json.load(open(path))["test-key"]["options"] == res.options
    finally:
        tune.apply_options(tune.DEFAULTS)
