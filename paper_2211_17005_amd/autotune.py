"""Autotuner of the persistent launches.

The free launch parameters of the regression are the team size -- how many workgroups train one
date together (the batch gradient summed across them, Adam sharded over them) -- and the wave
tiling of the BF16 kernels (which block of output tiles each wave owns, cva_mlp_cfg.tile).  More
workgroups per date shorten every SGD step but cost a cross-workgroup exchange per step and
leave fewer teams for the other dates; the best size depends on the number of dates, the batch,
the network, the number of epochs and the device; the best tiling depends on the width (register
pressure against operand reuse).  `regression_launch` times the actual fit with one and with
three epochs for each candidate size in the default tiling, then each tiling at the best size,
extrapolates linearly to the configured number of epochs (a fit has per-date costs that do not
scale with the epochs: statistics, the last epoch's losses when workgroups without a team
compute them) and keeps the fastest; the choice is cached in JSON keyed by (device, shape), so a
cached run is deterministic and costs nothing.  The cache file is `tuned.json` beside this
module unless HSIM_TUNE_CACHE names another path.
"""
from __future__ import annotations

import ctypes
import json
import os
import time

HERE = os.path.dirname(os.path.abspath(__file__))
CANDIDATES = (1, 2, 3, 4, 6, 8, 12, 16, 24, 32)


def cache_path() -> str:
    return os.environ.get("HSIM_TUNE_CACHE", os.path.join(HERE, "tuned.json"))


def _load() -> dict:
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _save(cache: dict) -> None:
    tmp = cache_path() + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, cache_path())


def device_key() -> str:
    import torch
    p = torch.cuda.get_device_properties(torch.cuda.current_device())
    return f"{getattr(p, 'gcnArchName', p.name)}/{p.multi_processor_count}cu"


def regression_key(cfg, n_dates: int, M: int) -> str:
    return (f"{device_key()}|regress|U{cfg.width}H{cfg.hidden}d{cfg.d_in}|batch{cfg.batch}"
            f"|epochs{cfg.epochs}|M{M}|dates{n_dates}|warm{cfg.warm_start}")


def _time_fit(hsim, torch, cfg, epochs: int, team: int, tile: int, dates, X, Y, seed: int, reps: int):
    """Min over `reps` runs of the wall time of one fit with `epochs`, `team`, `tile` (None if the
    configuration does not fit on the device)."""
    trial = hsim.MlpCfg(cfg.hidden, cfg.width, cfg.d_in, epochs, cfg.batch, cfg.lr, cfg.beta1,
                        cfg.beta2, cfg.eps, cfg.warm_start, cfg.init_tag, team, cfg.dtype, tile)
    if hsim.lib().cva_regress_workspace_bytes(ctypes.byref(trial), len(dates), int(X.shape[-1])) == 0:
        return None
    best = float("inf")
    for _ in range(reps):
        torch.cuda.synchronize()
        t = time.perf_counter()
        hsim.regress_fit(trial, dates, X, Y, seed=seed, want_loss=False)
        torch.cuda.synchronize()
        best = min(best, time.perf_counter() - t)
    return best


def _extrapolated(hsim, torch, cfg, team: int, tile: int, dates, X, Y, seed: int, reps: int):
    """t(1) + (E - 1) (t(3) - t(1)) / 2: the fit time at the configured E from one- and
    three-epoch fits (None if it does not fit)."""
    E = int(cfg.epochs)
    t1 = _time_fit(hsim, torch, cfg, 1, team, tile, dates, X, Y, seed, reps)
    if t1 is None or E == 1:
        return t1
    t3 = _time_fit(hsim, torch, cfg, 3, team, tile, dates, X, Y, seed, reps)
    return None if t3 is None else t1 + (E - 1) * (t3 - t1) / 2.0


def regression_launch(cfg, dates, X, Y, seed: int = 0, candidates=CANDIDATES, force: bool = False,
                      reps: int = 2) -> tuple:
    """(team size, wave tiling) for fitting `dates` of X / Y with `cfg` (a hsim.MlpCfg): the cached
    choice, or the team candidate with the least extrapolated fit time in the default tiling, then
    the fastest tiling at that team size (BF16 kernels only; the FP32 / FP64 form has one)."""
    import torch
    from . import hsim
    n_dates = len(dates)
    M = int(X.shape[-1])
    key = regression_key(cfg, n_dates, M)
    cache = _load()
    if key in cache and not force and "tile" in cache[key]:
        return int(cache[key]["team"]), int(cache[key]["tile"])
    chunks = -(-cfg.batch // 64)
    times = {}
    for team in candidates:
        if team > max(1, chunks):
            continue
        t = _extrapolated(hsim, torch, cfg, team, 0, dates, X, Y, seed, reps)
        if t is not None:
            times[team] = t
    if not times:
        raise RuntimeError("no team size fits on the device for this regression")
    team = min(times, key=lambda t: (times[t], t))
    tiles = {0: times[team]}
    if cfg.dtype == hsim.REG_BF16:
        for tile in range(1, hsim.MLP_TILES):
            t = _extrapolated(hsim, torch, cfg, team, tile, dates, X, Y, seed, reps)
            if t is not None:
                tiles[tile] = t
    tile = min(tiles, key=lambda t: (tiles[t], t))
    cache[key] = {"team": team, "tile": tile, "fit_ms": {str(k): round(v * 1e3, 3) for k, v in times.items()},
                  "tile_fit_ms": {str(k): round(v * 1e3, 3) for k, v in tiles.items()}}
    _save(cache)
    return team, tile


def regression_team(cfg, dates, X, Y, seed: int = 0, candidates=CANDIDATES, force: bool = False,
                    reps: int = 2) -> int:
    """The team size of regression_launch."""
    return regression_launch(cfg, dates, X, Y, seed, candidates, force, reps)[0]
