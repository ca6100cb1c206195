"""Writes the oracle's CVA_0 gradient on the ten-currency workload (test data, oracle only).

The differentiation form's market (10 economies, 9 FX rates, 8 counterparties, 500 swaps,
100 pricing dates x 25 Euler sub-steps) is simulated by the FP64 oracle on the first PATHS outer
paths; the smoothed CVA_0 estimator (the exact inner conditional expectation of the pathwise
loss, the intensity route of Section 4.2) and its central differences with common random
numbers are written for all 90 inputs (r0, FX0, lambda0, a, b, sigma_r, sigma_fx, kappa, theta,
nu), at the differentiation form's relative bump h = 1e-4 and at h = 1e-5.  The smoothed estimator
has kinks where an exposure (MtM)^+ crosses zero; a bump that carries a path across one moves
the difference quotient by O(h) on that input, so the two bumps show where that happened.

Run:    python tests/golden/make_adjoint_cfg2.py [--procs N]
Output: tests/golden/adjoint_cfg2_fd.txt ("name fd(1e-4) fd(1e-5)" per input, CVA_0 first).
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

PATHS = 512
HS = (1e-4, 1e-5)
OUT = os.path.join(HERE, "adjoint_cfg2_fd.txt")


def _workload():
    import workloads as wl
    return wl.differentiation_form(M=PATHS)


def _step(h, theta):
    return h * abs(theta) if theta != 0.0 else h


def _cva(job):
    """CVA_0 with input k bumped by sign * h |theta_k| (k < 0: the unbumped value)."""
    from oracle import model
    from oracle import sensitivities as osn
    k, sign, h = job
    w = _workload()
    base = osn.pack(w.market)
    v = base.copy()
    if k >= 0:
        v[k] += sign * _step(h, base[k])
    return k, sign, h, osn.cva0_smoothed(w, np.arange(PATHS), osn.unpack(w.market, v), model.fixed_rates(w))


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--procs", type=int, default=min(16, os.cpu_count() or 1))
    args = ap.parse_args(argv)
    from oracle import sensitivities as osn
    import multiprocessing as mp
    w = _workload()
    base = osn.pack(w.market)
    jobs = [(-1, 0, 0.0)] + [(k, s, h) for h in HS for k in range(base.size) for s in (+1, -1)]
    vals = {}
    t0 = time.time()
    os.environ["OMP_NUM_THREADS"] = "1"
    with mp.get_context("spawn").Pool(args.procs) as pool:
        for k, s, h, v in pool.imap_unordered(_cva, jobs):
            vals[(k, s, h)] = v
    names = osn.names(w.market)
    with open(OUT, "w") as f:
        f.write(f"# oracle CVA_0 (smoothed) and central differences with common random numbers at relative\n")
        f.write(f"# bumps h = {HS[0]:g} and {HS[1]:g}, first {PATHS} paths of the {w.name} workload;\n")
        f.write("# written by tests/golden/make_adjoint_cfg2.py\n")
        f.write(f"cva0 {vals[(-1, 0, 0.0)]:.17g}\n")
        for k in range(base.size):
            g = [(vals[(k, 1, h)] - vals[(k, -1, h)]) / (2.0 * _step(h, base[k])) for h in HS]
            f.write(f"{names[k]} {g[0]:.17g} {g[1]:.17g}\n")
    print(f"{OUT} in {time.time() - t0:.0f} s")


def load():
    """(cva0, names, gradient [inputs][bumps]) from the stored file."""
    names, vals, cva0 = [], [], None
    with open(OUT) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            k, *v = line.split()
            if k == "cva0":
                cva0 = float(v[0])
            else:
                names.append(k)
                vals.append([float(x) for x in v])
    return cva0, names, np.array(vals)


if __name__ == "__main__":
    main()
