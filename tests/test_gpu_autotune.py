"""The launch autotuner: a timed choice of the team size among the candidates that fit, then of
the kernels' wave tiling at that size, cached per (device, shape), so that a second call is
deterministic and does not time again."""
import json
import os

import numpy as np
import pytest

import workloads as wl

pytestmark = pytest.mark.gpu


def test_regression_launch_is_cached(lib, tmp_path, monkeypatch):
    import torch
    from paper_2211_17005_amd import autotune
    monkeypatch.setenv("HSIM_TUNE_CACHE", str(tmp_path / "tuned.json"))
    rng = np.random.default_rng(0)
    M, d = 8192, 5
    X = torch.as_tensor(rng.standard_normal((4, d, M)).astype(np.float32), device="cuda")
    Y = torch.as_tensor(np.abs(rng.standard_normal((4, M))).astype(np.float32), device="cuda")
    cfg = lib.mlp_cfg(wl.MLPConfig(hidden=2, width=128, epochs=3, batch=1024), d, M)
    team, tile = autotune.regression_launch(cfg, [1, 2, 3], X, Y, candidates=(1, 2, 4))
    assert team in (1, 2, 4) and tile in range(lib.MLP_TILES)
    cache = json.load(open(tmp_path / "tuned.json"))
    (key, entry), = cache.items()
    assert entry["team"] == team and set(entry["fit_ms"]) <= {"1", "2", "4"}
    assert entry["tile"] == tile and set(entry["tile_fit_ms"]) == {str(t) for t in range(lib.MLP_TILES)}
    # cached: the same answer without timing (candidates that could not run are not tried)
    assert autotune.regression_launch(cfg, [1, 2, 3], X, Y, candidates=()) == (team, tile)
    assert autotune.regression_team(cfg, [1, 2, 3], X, Y, candidates=()) == team
    # and the tuned launch trains like any other
    cfg.team, cfg.tile = team, tile
    model, loss, _ = lib.regress_fit(cfg, [1, 2, 3], X, Y)
    assert np.all(np.isfinite(loss.cpu().numpy()))
