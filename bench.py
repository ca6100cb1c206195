"""Benchmark of the hierarchical-simulation CVA path on one MI355X.

One step = one pass of the hot path over the 10-currency / 9-FX / 8-counterparty /
500-swap workload (100 pricing dates x 25 Euler sub-steps over 10y, M = 2^17 outer paths,
n_b = 128 inner default draws per path and counterparty), FP32 simulation with FP64
integrals:
  outer paths + pricing  ->  inner default draws  ->  targets and CVA_0
  [-> batched regression of the targets at every date]  [-> adjoint sensitivities]
with the stages that are built.  The metric is outer x inner path-steps per second:
M * n_b * n_dates / (seconds per step).

Prints one JSON line.  The CPU baseline (the FP64 oracle on a bounded sample of the
same workload, in worker processes on the host cores) runs before the GPU is touched.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import workloads as wl  # noqa: E402

# MI355X figures used for the roofline (AMD specifications and unit counts)
N_CU, CLOCK_HZ, LANES_PER_CU_CLK = 256, 2.4e9, 64
VALU_PEAK_OPS = N_CU * CLOCK_HZ * LANES_PER_CU_CLK          # 39.3e12 VALU lane-ops/s
HBM_PEAK = 8.0e12


def outer_ops_per_path(w) -> dict:
    """Algorithmic VALU operations of one outer path (one per elementary op; FMA = 1).

    Per Euler sub-step: Philox4x32-10 (10 rounds x (2 widening multiplies + 4 XOR)) per
    call of four words, 3 ops per uniform, 7 per Box-Muller pair (log, scale, sqrt, sin,
    cos, two products), d_W(d_W+1)/2 correlation FMAs, 2 per short rate, 4 per log-FX,
    11 per CIR intensity (two clamps, sqrt, 3 FMA, product, FP64 convert x2 + add + FMA),
    4 for the discount integral.  Per pricing date: per currency and future reset date one
    exp and 1 + C FMAs, plus per currency 3 + 4C ops for the floating leg, FX and bucket sums.
    """
    m = w.market
    n_e, C = m.n_ccy, m.n_cpty
    d_w = 2 * n_e - 1
    n_z = d_w + C
    calls = (n_z + 3) // 4
    sub = calls * (60 + 12 + 14) + d_w * (d_w + 1) // 2 + 2 * n_e + 4 * (n_e - 1) + 11 * C + 4
    S = w.grid.n_dates * w.grid.n_sub
    q = int(round(w.grid.n_dates * w.portfolio.delta / w.grid.horizon))
    P = int(np.max(w.portfolio.maturity))
    resets = sum(max(0, P - (i // q)) for i in range(w.grid.n_dates + 1))
    price = resets * n_e * (2 + C) + (w.grid.n_dates + 1) * n_e * (3 + 4 * C)
    return {"substep": sub, "total": S * sub + price}


def outer_bytes_per_path(w, real_bytes=4) -> int:
    """Algorithmic HBM bytes one outer path writes: features, I, Lambda, D."""
    n1 = w.grid.n_dates + 1
    d = wl.n_features(w)
    C = w.market.n_cpty
    return n1 * (d * real_bytes + 8 + C * 8 + C * real_bytes)


# ------------------------------------------------------------------------------- CPU baseline
def _oracle_chunk(args):
    name, kw, begin, count = args
    from oracle import pipeline
    w = wl.get(name, **kw)
    t = time.perf_counter()
    pipeline.simulate(w, path_begin=begin, count=count, chunk=count)
    return time.perf_counter() - t


def cpu_baseline(w, name, kw, paths_per_worker: int, workers: int):
    """The FP64 oracle on `workers * paths_per_worker` paths, one chunk per process."""
    import multiprocessing as mp
    ctx = mp.get_context("fork")          # runs before the GPU is initialised
    jobs = [(name, kw, i * paths_per_worker, paths_per_worker) for i in range(workers)]
    t0 = time.perf_counter()
    with ctx.Pool(workers) as pool:
        pool.map(_oracle_chunk, jobs)
    wall = time.perf_counter() - t0
    n_paths = workers * paths_per_worker
    rate = n_paths * w.n_b * w.grid.n_dates / wall
    return {"value": rate, "unit": "path-steps/s", "cores": workers, "kind": "oracle",
            "sample": f"{n_paths} outer paths x n_b={w.n_b} of the same workload "
                      f"(simulation, pricing, inner draws, targets), FP64 NumPy, "
                      f"{workers} processes, wall {wall:.1f} s"}


# ------------------------------------------------------------------------------- GPU step
def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--M", type=int, default=1 << 17)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-paths-per-worker", type=int, default=96)
    args = ap.parse_args()

    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; multi-GPU sharding is "
                                   "described in DESIGN.md but not implemented",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    name, kw = "cva_at_scale", {"M": args.M}
    w = wl.get(name, **kw)

    cpu = None
    if not args.no_cpu_baseline:
        workers = max(1, min(16, os.cpu_count() or 1))
        cpu = cpu_baseline(w, name, kw, args.cpu_paths_per_worker, workers)
        print(f"# cpu baseline: {cpu['value']:.4g} path-steps/s ({cpu['sample']})",
              file=sys.stderr, flush=True)

    import torch
    from paper_2211_17005_amd import hsim

    torch.cuda.set_device(0)
    prec = hsim.HSIM_FP32
    M, n1, C = w.M, w.grid.n_dates + 1, w.market.n_cpty
    d = wl.n_features(w)
    R = torch.float32
    stream = torch.cuda.current_stream()
    feats = torch.empty((n1, d, M), dtype=R, device="cuda")
    I = torch.empty((n1, M), dtype=torch.float64, device="cuda")
    Lam = torch.empty((n1, C, M), dtype=torch.float64, device="cuda")
    D = torch.empty((n1, C, M), dtype=R, device="cuda")
    cnt = torch.empty((n1, C, M), dtype=torch.int32, device="cuda")
    T = torch.empty((n1, M), dtype=R, device="cuda")
    cva0 = torch.empty(1, dtype=torch.float64, device="cuda")
    g = hsim.grid_struct(w.grid)
    wsb = hsim.lib().hsim_workspace_bytes(hsim.OP_TARGETS, None, hsim.ctypes.byref(g), M, prec)
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    fixed = hsim.fixed_rates(w.market, w.portfolio)
    km, kp = hsim.market_struct(w.market), hsim.portfolio_struct(w.portfolio, fixed)
    fm = hsim.feature_mode_of(w)
    L = hsim.lib()
    P = hsim._dptr
    by = hsim.ctypes.byref

    def step(ev=None):
        if ev is not None:
            ev[0].record(stream)
        hsim.check(L.hsim_outer_paths(by(km.struct), by(kp.struct), by(g), w.seed, 0, M, prec, fm,
                                      P(feats), P(I), P(Lam), P(D), None, hsim._stream()))
        if ev is not None:
            ev[1].record(stream)
        hsim.check(L.hsim_inner_defaults(by(g), C, w.seed, 0, M, w.n_b, None, 64, P(Lam), P(cnt),
                                         None, 0, hsim._stream()))
        if ev is not None:
            ev[2].record(stream)
        hsim.check(L.hsim_targets_cva(by(g), C, M, w.n_b, None, 64, prec, P(I), P(D), P(cnt),
                                      P(T), P(cva0), P(ws), wsb, hsim._stream()))
        if ev is not None:
            ev[3].record(stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(args.steps)]
    t0 = time.perf_counter()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    start.record(stream)
    for k in range(args.steps):
        step(evs[k])
    end.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = start.elapsed_time(end) / args.steps
    outer_ms = float(np.mean([e[0].elapsed_time(e[1]) for e in evs]))
    inner_ms = float(np.mean([e[1].elapsed_time(e[2]) for e in evs]))
    targ_ms = float(np.mean([e[2].elapsed_time(e[3]) for e in evs]))

    path_steps = M * w.n_b * w.grid.n_dates
    value = path_steps / (ms_step / 1e3)
    ops = outer_ops_per_path(w)["total"] * M
    achieved = ops / (outer_ms / 1e3)
    rec = {
        "metric": "outer x inner path-steps/s (hierarchical CVA simulation, 1 GPU)",
        "value": value,
        "unit": "path-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 (f64 integrals)",
        "data": "synthetic (seeded model parameters, LKJ(2) correlation, random swap book)",
        "config": {"workload": w.name, "n_ccy": w.market.n_ccy, "n_cpty": C,
                   "n_swaps": w.portfolio.n_swaps, "n_dates": w.grid.n_dates,
                   "n_sub": w.grid.n_sub, "M": M, "n_b": w.n_b,
                   "stages": ["outer+pricing", "inner defaults", "targets+CVA_0"]},
        "stage_ms": {"outer_kernel": outer_ms, "inner_kernel": inner_ms,
                     "targets_kernels": targ_ms},
        "roofline": {"bound": "alu", "kernel": "outer_kernel<float,10,8>",
                     "achieved": achieved / 1e12, "peak": VALU_PEAK_OPS / 1e12,
                     "unit": "T VALU lane-ops/s", "frac": achieved / VALU_PEAK_OPS,
                     "traffic": None},
        "cva0": cva0.item(),
        "cpu_baseline": cpu,
        "wall_s": wall,
    }
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
