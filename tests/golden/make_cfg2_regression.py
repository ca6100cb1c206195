"""Writes the oracle's regression case at the precision-form shape (test data, oracle only).

The ten-currency / eight-counterparty workload (Section 4.3 case: 10 economies, 8 clients,
500 swaps, 100 pricing dates, 25 Euler sub-steps) at M = 2^17 outer paths and n_b = 128 inner
draws is simulated by the FP64 oracle; at the dates in DATES its 29 regression inputs (27 market
factors, the discount integral and the summed intensity integrals) and its CVA targets are
rounded to FP32 (the library's input type), and the oracle's BaseAlg (Algorithm 1) fits them in
FP64 from the common initial draw (3 hidden layers of 128 units, batch 8192, 50 epochs).  Saved:
inputs, targets, the FP64 predictions on the same rows and the FP64 loss histories, and the same
for HOLD held-out paths [M, M + HOLD) (inputs, targets, the FP64 fits' predictions).

Run:  python tests/golden/make_cfg2_regression.py [--procs N]
Output: tests/golden/cache/cfg2_regression_M131072_hold16384.npz (about 70 MB, not committed).
"""
from __future__ import annotations

import argparse
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

DATES = (10, 25, 50, 90)
M = 1 << 17
HOLD = 1 << 14
CHUNK = 2048
OUT = os.path.join(HERE, "cache", f"cfg2_regression_M{M}_hold{HOLD}.npz")


def _sim_chunk(c0: int):
    import workloads as wl
    from oracle import pipeline
    w = wl.precision_form(M=M)
    r = pipeline.simulate(w, path_begin=c0, count=min(CHUNK, M + HOLD - c0), chunk=512)
    d = list(DATES)
    return c0, r["features"][d].astype(np.float32), r["T"][d].astype(np.float32)


def _fit(args):
    j, X, y, Xh = args
    import workloads as wl
    from oracle import regression as org
    mlp = wl.precision_form(M=M).mlp
    Xd = X.astype(np.float64).T
    fit = org.fit_date(Xd, y.astype(np.float64), mlp, org.init_net(Xd.shape[1], mlp.hidden, mlp.width,
                                                                  wl.precision_form(M=M).seed), mlp.batch)
    return j, org.predict(fit, Xd), np.array(fit.losses), org.predict(fit, Xh.astype(np.float64).T)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--procs", type=int, default=min(16, os.cpu_count() or 1))
    args = ap.parse_args(argv)
    import multiprocessing as mp
    t0 = time.time()
    n_feat = 29
    X = np.empty((len(DATES), n_feat, M + HOLD), np.float32)
    T = np.empty((len(DATES), M + HOLD), np.float32)
    os.environ["OMP_NUM_THREADS"] = "1"
    with mp.get_context("spawn").Pool(args.procs) as pool:
        for c0, f, t in pool.imap_unordered(_sim_chunk, range(0, M + HOLD, CHUNK)):
            X[:, :, c0:c0 + f.shape[2]] = f
            T[:, c0:c0 + t.shape[1]] = t
    print(f"simulated {M + HOLD} paths in {time.time() - t0:.0f} s", flush=True)
    pred = np.empty((len(DATES), M))
    pred_h = np.empty((len(DATES), HOLD))
    losses = [None] * len(DATES)
    os.environ["OMP_NUM_THREADS"] = str(max(1, args.procs // len(DATES)))
    with mp.get_context("spawn").Pool(min(args.procs, len(DATES))) as pool:
        jobs = [(j, X[j, :, :M], T[j, :M], X[j, :, M:]) for j in range(len(DATES))]
        for j, p, l, ph in pool.imap_unordered(_fit, jobs):
            pred[j] = p
            losses[j] = l
            pred_h[j] = ph
    print(f"fitted {len(DATES)} dates in {time.time() - t0:.0f} s", flush=True)
    os.makedirs(os.path.dirname(OUT), exist_ok=True)
    np.savez(OUT, dates=np.array(DATES), X=np.ascontiguousarray(X[:, :, :M]), T=np.ascontiguousarray(T[:, :M]),
             pred64=pred, loss64=np.stack(losses), X_hold=np.ascontiguousarray(X[:, :, M:]),
             T_hold=np.ascontiguousarray(T[:, M:]), pred64_hold=pred_h)
    print(OUT)


if __name__ == "__main__":
    main()
