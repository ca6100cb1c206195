"""CVA_0 sensitivities by central finite differences with common random numbers (oracle).

The indicator estimator T^k_0 is piecewise constant in the intensity integrals
Lambda^c, so its pathwise derivative with respect to the credit parameters is zero
almost surely.  The quantity differentiated is therefore the smoothed estimator
    CVA_0 = mean_k sum_c sum_{j>=1} D^c_j (exp(-Lambda^c_{j-1}) - exp(-Lambda^c_j)),
i.e. the exact inner conditional expectation of the pathwise loss (the
intensity route that Section 4.2 calls the minimal-variance CVA learner), whose
expectation equals that of the indicator estimator.

Parameter vector (in this order): r0[n_e], fx0[n_e-1], lambda0[C], a[n_e], b[n_e],
sigma_r[n_e], sigma_fx[n_e-1], kappa[C], theta[C], nu[C].  The swap book's fixed
rates are held at their base values while parameters are bumped.
"""
from __future__ import annotations

from dataclasses import replace

import numpy as np

from . import inner, model

FIELDS = ("r0", "fx0", "lambda0", "a", "b", "sigma_r", "sigma_fx", "kappa", "theta", "nu")


def pack(m) -> np.ndarray:
    return np.concatenate([np.asarray(getattr(m, f), dtype=np.float64) for f in FIELDS])


def names(m):
    out = []
    for f in FIELDS:
        out += [f"{f}[{i}]" for i in range(len(getattr(m, f)))]
    return out


def unpack(m, vec: np.ndarray):
    kw, o = {}, 0
    for f in FIELDS:
        k = len(getattr(m, f))
        kw[f] = np.array(vec[o:o + k], dtype=np.float64)
        o += k
    return replace(m, **kw)


def cva0_smoothed(w, paths, market=None, fixed=None, chunk: int = 512) -> float:
    m = w.market if market is None else market
    fixed = model.fixed_rates(w) if fixed is None else fixed
    total = 0.0
    paths = np.asarray(paths)
    for s in range(0, paths.shape[0], chunk):
        p = paths[s:s + chunk]
        outer = model.simulate_outer(w, p, m)
        mt = model.mtm(w, outer, fixed, m)
        D = model.exposure(w, outer, mt, m)                 # [n+1, P, C]
        surv = np.exp(-outer.Lam)
        prob = surv[:-1] - surv[1:]                          # [n, P, C]
        total += float((D[1:] * prob).sum())
    return total / paths.shape[0]


def fd_gradient(w, paths, h: float = 1e-4, index=None, chunk: int = 512) -> np.ndarray:
    """Central differences, relative bump h*|theta| (absolute h where theta = 0)."""
    base = pack(w.market)
    fixed = model.fixed_rates(w)
    idx = range(base.shape[0]) if index is None else index
    g = np.zeros(base.shape[0])
    for k in idx:
        step = h * abs(base[k]) if base[k] != 0.0 else h
        up, dn = base.copy(), base.copy()
        up[k] += step
        dn[k] -= step
        fu = cva0_smoothed(w, paths, unpack(w.market, up), fixed, chunk)
        fd = cva0_smoothed(w, paths, unpack(w.market, dn), fixed, chunk)
        g[k] = (fu - fd) / (2.0 * step)
    return g


def indicator_cva0(w, paths, n_b=None) -> float:
    """Indicator-estimator CVA_0 on the same paths (for the expectation check)."""
    m = w.market
    fixed = model.fixed_rates(w)
    outer = model.simulate_outer(w, paths, m)
    mt = model.mtm(w, outer, fixed, m)
    u = inner.inner_draws(w, paths, n_b)
    js = inner.default_dates(outer.Lam, u)
    xi = inner.pathwise_loss(outer.I, mt, m.lgd, js)
    return float(inner.targets(xi)[0].mean())
