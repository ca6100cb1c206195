"""Branched re-simulation: nested and twin Monte Carlo estimates of the conditional CVA
(FP64 oracle).

TEST INFRASTRUCTURE ONLY (see the package header).

From the state of outer path k at a pricing date t_i, B conditionally independent
continuations b = 0..B-1 of the market are simulated (branch normals after t_i, the
outer path's own normals before).  Each continuation gives the intensity-form sample

    xi^{k,b} = exp(I_i) sum_{j>i} sum_c D^{c,b}_j (exp(-Lambda^{c,b}_{j-1}) - exp(-Lambda^{c,b}_j)),

whose conditional mean given the state at t_i is the CVA of eq. CVAint (read, as for the
intensity targets, with the exact survival increments of the fine-grid Lambda).  From
these samples and a prediction phi^k of that conditional mean:

  * the nested Monte Carlo estimate (Section 4.3's benchmark) nu^k = mean_b xi^{k,b};
  * the twin Monte Carlo L^2 error (Section 3.3, e:val1 with e:val2), generalised from two
    copies to all ordered pairs of distinct continuations:
        E[(phi - CVA_i)^2] = E[phi^2 - 2 phi nu + U],
        U^k = sum_{b != b'} xi^{k,b} xi^{k,b'} / (B (B - 1)),
    which for B = 2 is exactly phi^2 - (xi^1 + xi^2) phi + xi^1 xi^2.
"""
from __future__ import annotations

import numpy as np

from . import inner, model

# order of the summary statistics of twin_errors (and of the GPU reduction)
STATS = ("cva_mean", "cva_sq_nested", "cva_sq", "mse_nested", "mse_twin", "phi_mean")


def branch_targets(w, paths, date: int, n_branch: int, market=None, fixed=None) -> np.ndarray:
    """xi [B, P]: the intensity-form sample of every continuation b of every outer path."""
    m = w.market if market is None else market
    fixed = model.fixed_rates(w, m) if fixed is None else fixed
    paths = np.asarray(paths, dtype=np.int64)
    P = paths.shape[0]
    lane_path = np.tile(paths, n_branch)                 # lane = b * P + p
    lane_branch = np.repeat(np.arange(n_branch), P)
    outer = model.simulate_outer(w, lane_path, m, branch=lane_branch, branch_date=date)
    mt = model.mtm(w, outer, fixed, m)
    mu, _ = inner.conditional_moments(outer.I, outer.Lam, mt, m.lgd)
    return mu[date].reshape(n_branch, P)


def twin_errors(phi, xi) -> dict:
    """Path averages of the nested / twin Monte Carlo quantities (names in STATS).

    phi [P] predictions at the branching date, xi [B, P] continuation samples, B >= 2.
      cva_mean       mean_k nu^k                      (nested CVA, E[CVA_i])
      cva_sq_nested  mean_k (nu^k)^2                  (biased by E[Var]/B)
      cva_sq         mean_k U^k                       (unbiased for E[CVA_i^2])
      mse_nested     mean_k (phi^k - nu^k)^2          (biased by E[Var]/B)
      mse_twin       mean_k (phi^k)^2 - 2 phi^k nu^k + U^k   (unbiased, e:val1)
      phi_mean       mean_k phi^k
    """
    phi = np.asarray(phi, dtype=np.float64)
    xi = np.asarray(xi, dtype=np.float64)
    B = xi.shape[0]
    if B < 2:
        raise ValueError("the twin estimator needs at least two continuations")
    nu = xi.mean(axis=0)
    S1 = xi.sum(axis=0)
    S2 = (xi * xi).sum(axis=0)
    U = (S1 * S1 - S2) / (B * (B - 1))
    vals = (nu.mean(), (nu * nu).mean(), U.mean(), ((phi - nu) ** 2).mean(),
            (phi * phi - 2.0 * phi * nu + U).mean(), phi.mean())
    return dict(zip(STATS, (float(v) for v in vals)))
