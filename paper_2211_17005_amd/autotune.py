"""Autotuner of the persistent launches.

The one free launch parameter that matters is the regression team size: how many workgroups
train one date together (the batch gradient summed across them, Adam sharded over them).  More
workgroups per date shorten every SGD step but cost a cross-workgroup exchange per step and
leave fewer teams for the other dates; the best size depends on the number of dates, the batch,
the network, the number of epochs and the device.  `regression_team` times the actual fit with
one and with three epochs for each candidate size, extrapolates linearly to the configured
number of epochs (a fit has per-date costs that do not scale with the epochs: statistics, the
last epoch's losses when workgroups without a team compute them) and keeps the fastest; the
choice is cached in JSON keyed by (device, shape), so a cached run is deterministic and costs
nothing.  The cache file is `tuned.json` beside this
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


def regression_team(cfg, dates, X, Y, seed: int = 0, candidates=CANDIDATES, force: bool = False,
                    reps: int = 2) -> int:
    """Team size for fitting `dates` of X / Y with `cfg` (a hsim.MlpCfg): the cached choice, or
    the candidate with the least extrapolated time t(1) + (E - 1) (t(3) - t(1)) / 2 of the real
    fit (each timing the min of `reps` runs)."""
    import torch
    from . import hsim
    n_dates = len(dates)
    M = int(X.shape[-1])
    key = regression_key(cfg, n_dates, M)
    cache = _load()
    if key in cache and not force:
        return int(cache[key]["team"])
    chunks = -(-cfg.batch // 64)
    E = int(cfg.epochs)
    times = {}
    for team in candidates:
        if team > max(1, chunks):
            continue
        t_e = {}
        for epochs in ((1, 3) if E > 1 else (1,)):
            trial = hsim.MlpCfg(cfg.hidden, cfg.width, cfg.d_in, epochs, cfg.batch, cfg.lr, cfg.beta1,
                                cfg.beta2, cfg.eps, cfg.warm_start, cfg.init_tag, team, cfg.dtype)
            if hsim.lib().cva_regress_workspace_bytes(ctypes.byref(trial), n_dates, M) == 0:
                break                                  # does not fit on the device
            best = float("inf")
            for _ in range(reps):
                torch.cuda.synchronize()
                t = time.perf_counter()
                hsim.regress_fit(trial, dates, X, Y, seed=seed, want_loss=False)
                torch.cuda.synchronize()
                best = min(best, time.perf_counter() - t)
            t_e[epochs] = best
        if 1 not in t_e or (E > 1 and 3 not in t_e):
            continue
        times[team] = t_e[1] + (E - 1) * (t_e[3] - t_e[1]) / 2.0 if E > 1 else t_e[1]
    if not times:
        raise RuntimeError("no team size fits on the device for this regression")
    team = min(times, key=lambda t: (times[t], t))
    cache[key] = {"team": team, "fit_ms": {str(k): round(v * 1e3, 3) for k, v in times.items()}}
    _save(cache)
    return team
